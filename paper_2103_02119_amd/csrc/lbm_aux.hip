// Conversion, output and reduction kernels of the library (host-facing
// FP64 fields and populations, the smoothing step's average, the local
// stress, the deterministic FP64 sums and residuals) and the streaming copy
// that measures the achievable HBM bandwidth.
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

// ------------------------------------------------------------ conversions

// Equilibrium in product form: feq_k = rho Px(cx_k) Py(cy_k) with
// Px(0) = 1 - s - ux^2, Px(+-1) = (s + ux^2 +- ux)/2,
// Py(0) = 1 - (s + uy^2)/a^2, Py(+-1) = (s + uy^2 +- a uy)/(2 a^2);
// this is T^{-1} F(-u) applied to Eq. 49 without corrections.
__device__ __forceinline__ double px_of(int cx, double s, double u) {
    return cx == 0 ? 1.0 - s - u * u : 0.5 * (s + u * u + cx * u);
}
__device__ __forceinline__ double py_of(int cy, double s, double a, double u) {
    const double ia2 = 1.0 / (a * a);
    return cy == 0 ? 1.0 - (s + u * u) * ia2 : 0.5 * (s + u * u + cy * a * u) * ia2;
}

template <typename S>
__global__ void init_feq_kernel(S *__restrict__ dst, const double *__restrict__ rho,
                                const double *__restrict__ ux, const double *__restrict__ uy,
                                const Geometry G, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        const long long o = static_cast<long long>(j) * G.pitch + x;
        const bool solid = G.mask && G.mask[o];  // solid nodes take the rest state
        const double r = (rho && !solid) ? rho[idx] : H.rho0;
        const double vx = (ux && !solid) ? ux[idx] : 0.0, vy = (uy && !solid) ? uy[idx] : 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double f = r * px_of(cx_of(k), H.s, vx) * py_of(cy_of(k), H.s, H.a, vy);
            if (H.dev) f -= H.rho0 * H.wrest[k];
            dst[k * G.plane + o] = static_cast<S>(f);
        }
    }
}

template <typename S>
__global__ void set_pop_kernel(S *__restrict__ dst, const double *__restrict__ f,
                               const Geometry G, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        const long long o = static_cast<long long>(j) * G.pitch + x;
        const bool solid = G.mask && G.mask[o];  // solid nodes take the rest state
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double v = solid ? H.rho0 * H.wrest[k] : f[k * n + idx];
            if (H.dev) v -= H.rho0 * H.wrest[k];
            dst[k * G.plane + o] = static_cast<S>(v);
        }
    }
}

template <typename S, bool PULL>
__global__ void get_pop_kernel(const S *__restrict__ src, double *__restrict__ f,
                               const Geometry G, const Consts<double> K, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        double f9[9];
        load_node<S, double, PULL>(src, G, K, row_info(j, G), col_info(x, G), f9);
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k * n + idx] = f9[k] + (H.dev ? H.rho0 * H.wrest[k] : 0.0);
    }
}

// f = (state n + state n-1) / 2 in FP64 [9][n] (full populations), from the
// current buffer (pull form PC) and the previous one (pull form PP)
template <typename S, bool PC, bool PP>
__global__ void avg_states_kernel(const S *__restrict__ cur, const S *__restrict__ prev,
                                  double *__restrict__ f, const Geometry G,
                                  const Consts<double> K, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        const RowInfo ri = row_info(j, G);
        const ColInfo ci = col_info(x, G);
        double a9[9], b9[9];
        load_node<S, double, PC>(cur, G, K, ri, ci, a9);
        load_node<S, double, PP>(prev, G, K, ri, ci, b9);
#pragma unroll
        for (int k = 0; k < 9; ++k)
            f[k * n + idx] = 0.5 * (a9[k] + b9[k]) + (H.dev ? H.rho0 * H.wrest[k] : 0.0);
    }
}

// rho, u of one node from its pre-collision values, in FP64
__device__ __forceinline__ void macro_of(const double (&f9)[9], const HostSide &H, double &r,
                                         double &vx, double &vy) {
    double s = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        s += f9[k];
        jx += cx_of(k) * f9[k];
        jy += cy_of(k) * f9[k];
    }
    r = s + (H.dev ? H.rho0 : 0.0);
    vx = (jx + 0.5 * H.Fx) / r;
    vy = (H.a * jy + 0.5 * H.Fy) / r;
}

template <typename S, bool PULL>
__global__ void moments_kernel(const S *__restrict__ src, double *__restrict__ rho,
                               double *__restrict__ ux, double *__restrict__ uy,
                               const Geometry G, const Consts<double> K, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        double f9[9], r, vx, vy;
        load_node<S, double, PULL>(src, G, K, row_info(j, G), col_info(x, G), f9);
        macro_of(f9, H, r, vx, vy);
        rho[idx] = r;
        ux[idx] = vx;
        uy[idx] = vy;
    }
}

// Density of the neighbour of (x, j) that the density gradient uses: across
// a periodic face it wraps; across a wall, or onto a solid node, it is the
// node's own density.
__device__ __forceinline__ double nb_rho(const double *__restrict__ rho, const Geometry &G, int x,
                                         int j, int dx, int dy) {
    int xn = x + dx, jn = j + dy;
    if (xn < 0) {
        if (G.bc[kXmin] != kPeriodic) return rho[static_cast<long long>(j) * G.nx + x];
        xn = G.nx - 1;
    } else if (xn >= G.nx) {
        if (G.bc[kXmax] != kPeriodic) return rho[static_cast<long long>(j) * G.nx + x];
        xn = 0;
    }
    if (jn < 0) {
        if (G.bc[kYmin] != kPeriodic) return rho[static_cast<long long>(j) * G.nx + x];
        jn = G.ny - 1;
    } else if (jn >= G.ny) {
        if (G.bc[kYmax] != kPeriodic) return rho[static_cast<long long>(j) * G.nx + x];
        jn = 0;
    }
    if (G.mask && G.mask[static_cast<long long>(jn) * G.pitch + xn])
        return rho[static_cast<long long>(j) * G.nx + x];
    return rho[static_cast<long long>(jn) * G.nx + xn];
}

// Local viscous stress of every node, in FP64, from its pre-collision
// populations and the densities of its neighbours: the strain rate of
// Eq. 37-39 (d_x u_x, d_y u_y from the second-order non-equilibrium moments
// with the density-gradient terms of Eq. 40; the shear rate from m_5 alone,
// its correction being zero by Eq. 27), then the viscous terms of Eq. 30-31
// with nu and zeta of Eq. 32-33.  Solid nodes get 0.
template <typename S, bool PULL>
__global__ void stress_kernel(const S *__restrict__ src, const double *__restrict__ rho,
                              double *__restrict__ sxx, double *__restrict__ syy,
                              double *__restrict__ sxy, const Geometry G, const Consts<double> K,
                              const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    const double nu4 = K.s * K.k4, zeta = K.s * K.k3, nu5 = K.s * (1.0 / K.w[5] - 0.5);
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(idx % G.nx), j = static_cast<int>(idx / G.nx);
        if (G.mask && G.mask[static_cast<long long>(j) * G.pitch + x]) {
            sxx[idx] = syy[idx] = sxy[idx] = 0.0;
            continue;
        }
        double f9[9], r, ux, uy;
        load_node<S, double, PULL>(src, G, K, row_info(j, G), col_info(x, G), f9);
        macro_of(f9, H, r, ux, uy);
        // raw second moments of the stored values (deviations from rho0 w_k
        // when H.dev: the rest state's own m_3 = 2 cs2 rho0, m_4 = m_5 = 0)
        double r00 = 0.0, r20 = 0.0, r02 = 0.0, r11 = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            r00 += f9[k];
            r20 += cx_of(k) * cx_of(k) * f9[k];
            r02 += cy_of(k) * cy_of(k) * f9[k];
            r11 += cx_of(k) * cy_of(k) * f9[k];
        }
        const double ux2 = ux * ux, uy2 = uy * uy;
        const double Q3 = (r20 + K.a2 * r02) - 2.0 * K.s * r00 - r * (ux2 + uy2);
        const double Q4 = (r20 - K.a2 * r02) - r * (ux2 - uy2);
        const double N5 = K.a * r11 - r * ux * uy;
        const double gx = 0.5 * (nb_rho(rho, G, x, j, 1, 0) - nb_rho(rho, G, x, j, -1, 0));
        const double gy = K.half_inv_a * (nb_rho(rho, G, x, j, 0, 1) - nb_rho(rho, G, x, j, 0, -1));
        const double tx = K.e1 * ux * gx, ty = K.e2 * uy * gy;
        const double M3 = Q3 - tx - ty, M4 = Q4 - tx + ty;
        const double b1 = K.b1c + 1.5 * ux2, b2 = K.b2c + 1.5 * uy2;
        const double c1 = K.c1c + 1.5 * ux2, c2 = K.c2c - 1.5 * uy2;
        const double idet = 1.0 / (r * (b1 * c2 - c1 * b2));
        const double X = (c2 * M3 - b2 * M4) * idet;  // d ux / dx
        const double Y = (b1 * M4 - c1 * M3) * idet;  // d uy / dy
        const double shear = -N5 * K.w[5] / (r * K.s);  // d uy / dx + d ux / dy
        const double div = X + Y;
        sxx[idx] = r * (nu4 * (2.0 * X - div) + zeta * div);
        syy[idx] = r * (nu4 * (2.0 * Y - div) + zeta * div);
        sxy[idx] = r * nu5 * shear;
    }
}

// ------------------------------------------------------------ reductions

// Deterministic FP64 block sum of N values: wavefront shuffle tree, then
// the wavefront totals in a fixed order.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *out) {
    __shared__ double part[kReduceBlock / kWave][N];
#pragma unroll
    for (int q = 0; q < N; ++q)
        for (int off = kWave / 2; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    if (lane == 0)
        for (int q = 0; q < N; ++q) part[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < N; ++q) {
            double t = 0.0;
            for (int i = 0; i < kReduceBlock / kWave; ++i) t += part[i][q];
            out[q] = t;
        }
    }
}

// Column and row of node idx (row-major, nx per row); 32-bit division when
// the lattice has fewer than 2^32 nodes, which is the uniform case.
__device__ __forceinline__ void node_xy(long long idx, int nx, bool narrow, int &x, int &j) {
    if (narrow) {
        const unsigned u = static_cast<unsigned>(idx), q = u / static_cast<unsigned>(nx);
        j = static_cast<int>(q);
        x = static_cast<int>(u - q * static_cast<unsigned>(nx));
    } else {
        j = static_cast<int>(idx / nx);
        x = static_cast<int>(idx - static_cast<long long>(j) * nx);
    }
}

template <typename S, bool PULL>
__global__ void __launch_bounds__(kReduceBlock)
sums_kernel(const S *__restrict__ src, double *__restrict__ partials, const Geometry G,
            const Consts<double> K, const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool narrow = n <= 0xffffffffLL;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        int x, j;
        node_xy(idx, G.nx, narrow, x, j);
        if (G.mask && G.mask[static_cast<long long>(j) * G.pitch + x]) continue;  // fluid only
        double f9[9], r, vx, vy;
        load_node<S, double, PULL>(src, G, K, row_info(j, G), col_info(x, G), f9);
        macro_of(f9, H, r, vx, vy);
        acc[0] += r;
        acc[1] += r * vx;
        acc[2] += r * vy;
        if (!isfinite(r) || !isfinite(vx) || !isfinite(vy)) acc[3] = 1.0;
    }
    block_sum(acc, partials + 4 * blockIdx.x);
}

template <typename SC, typename SP, bool PC, bool PP>
__global__ void __launch_bounds__(kReduceBlock)
residual_kernel(const SC *__restrict__ cur, const SP *__restrict__ prev,
                double *__restrict__ partials, const Geometry G, const Consts<double> K,
                const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool narrow = n <= 0xffffffffLL;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        int x, j;
        node_xy(idx, G.nx, narrow, x, j);
        if (G.mask && G.mask[static_cast<long long>(j) * G.pitch + x]) continue;  // fluid only
        const RowInfo ri = row_info(j, G);
        const ColInfo ci = col_info(x, G);
        double f9[9], r, vx, vy, r0, wx, wy;
        load_node<SC, double, PC>(cur, G, K, ri, ci, f9);
        macro_of(f9, H, r, vx, vy);
        load_node<SP, double, PP>(prev, G, K, ri, ci, f9);
        macro_of(f9, H, r0, wx, wy);
        const double dx = vx - wx, dy = vy - wy;
        acc[0] += dx * dx + dy * dy;
        acc[1] += vx * vx + vy * vy;
        if (!isfinite(vx) || !isfinite(vy) || !isfinite(wx) || !isfinite(wy)) acc[3] = 1.0;
    }
    block_sum(acc, partials + 4 * blockIdx.x);
}

// The residual and the conservation sums of one time level in one pass over
// the two buffers: values 0..3 accumulate as in residual_kernel, 4..7 as in
// sums_kernel, node by node in the same order, so each total is the one the
// separate kernels give.  Held to 64 VGPRs (eight wavefronts per SIMD):
// measured on the 2048 x 8192 lattice, 458 against 590 us in FP32 storage and
// 571 against 604 us in FP64 with the compiler's own choice (80-95 VGPRs),
// despite a few spilled registers.
template <typename S, bool PC, bool PP>
__global__ void __launch_bounds__(kReduceBlock, 8)
check_kernel(const S *__restrict__ cur, const S *__restrict__ prev,
             double *__restrict__ partials, const Geometry G, const Consts<double> K,
             const HostSide H) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool narrow = n <= 0xffffffffLL;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < n;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        int x, j;
        node_xy(idx, G.nx, narrow, x, j);
        if (G.mask && G.mask[static_cast<long long>(j) * G.pitch + x]) continue;  // fluid only
        const RowInfo ri = row_info(j, G);
        const ColInfo ci = col_info(x, G);
        double f9[9], r, vx, vy, r0, wx, wy;
        load_node<S, double, PC>(cur, G, K, ri, ci, f9);
        macro_of(f9, H, r, vx, vy);
        load_node<S, double, PP>(prev, G, K, ri, ci, f9);
        macro_of(f9, H, r0, wx, wy);
        const double dx = vx - wx, dy = vy - wy;
        acc[0] += dx * dx + dy * dy;
        acc[1] += vx * vx + vy * vy;
        if (!isfinite(vx) || !isfinite(vy) || !isfinite(wx) || !isfinite(wy)) acc[3] = 1.0;
        acc[4] += r;
        acc[5] += r * vx;
        acc[6] += r * vy;
        if (!isfinite(r) || !isfinite(vx) || !isfinite(vy)) acc[7] = 1.0;
    }
    block_sum(acc, partials + 8 * blockIdx.x);
}

// sums the per-block partials (N per block) in a fixed order; the NaN flags
// (every fourth value) are or-ed (max)
template <int N>
__global__ void __launch_bounds__(kReduceBlock)
finalize_kernel(const double *__restrict__ partials, int nparts, double *__restrict__ out) {
    double acc[N];
#pragma unroll
    for (int q = 0; q < N; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const double v = partials[N * i + q];
            acc[q] = (q & 3) == 3 ? fmax(acc[q], v) : acc[q] + v;
        }
    }
    // flag: any non-zero survives the sum as non-zero
    block_sum(acc, out);
}

// Batched residual: one workgroup per reduction item (a run of nodes of one
// case), then one workgroup per case sums that case's item partials in a
// fixed order, so every case's result is deterministic.
template <typename S, bool PC, bool PP>
__device__ __forceinline__ void batch_residual_item(const S *cur, const S *prev, const Geometry &G,
                                                    const Consts<double> &K, const HostSide &H,
                                                    int start, int count, double (&acc)[4]) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const int idx = start + i;
        const int x = idx % G.nx, j = idx / G.nx;
        if (G.mask && G.mask[static_cast<long long>(j) * G.pitch + x]) continue;  // fluid only
        const RowInfo ri = row_info(j, G);
        const ColInfo ci = col_info(x, G);
        double f9[9], r, vx, vy, r0, wx, wy;
        load_node<S, double, PC>(cur, G, K, ri, ci, f9);
        macro_of(f9, H, r, vx, vy);
        load_node<S, double, PP>(prev, G, K, ri, ci, f9);
        macro_of(f9, H, r0, wx, wy);
        const double dx = vx - wx, dy = vy - wy;
        acc[0] += dx * dx + dy * dy;
        acc[1] += vx * vx + vy * vy;
        if (!isfinite(vx) || !isfinite(vy) || !isfinite(wx) || !isfinite(wy)) acc[3] = 1.0;
    }
}

template <typename S>
__global__ void __launch_bounds__(kReduceBlock)
batch_residual_kernel(const S *__restrict__ buf0, const S *__restrict__ buf1,
                      const BatchRed *__restrict__ items, const BatchCase *__restrict__ cases,
                      const Geometry *__restrict__ geoms, const Consts<double> *__restrict__ Kd,
                      const HostSide *__restrict__ Hs, double *__restrict__ partials) {
    const BatchRed it = items[blockIdx.x];
    const int c = it.c;
    const Geometry &G = geoms[c];
    const Consts<double> &K = Kd[c];
    const HostSide &H = Hs[c];
    const long long off = cases[c].off;
    const S *cur = (cases[c].cur ? buf1 : buf0) + off;
    const S *prev = (cases[c].cur ? buf0 : buf1) + off;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    switch (it.flags & 3) {
    case 0: batch_residual_item<S, false, false>(cur, prev, G, K, H, it.start, it.count, acc); break;
    case 1: batch_residual_item<S, true, false>(cur, prev, G, K, H, it.start, it.count, acc); break;
    case 2: batch_residual_item<S, false, true>(cur, prev, G, K, H, it.start, it.count, acc); break;
    default: batch_residual_item<S, true, true>(cur, prev, G, K, H, it.start, it.count, acc); break;
    }
    block_sum(acc, partials + 4 * blockIdx.x);
}

// out[4 c ..] = fixed-order sum of the partials of items first[c] .. first[c] + count[c] - 1
__global__ void __launch_bounds__(kReduceBlock)
batch_finalize_kernel(const double *__restrict__ partials, const int *__restrict__ first,
                      const int *__restrict__ count, double *__restrict__ out) {
    const int c = blockIdx.x;
    const int f = first[c], n = count[c];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double *p = partials + 4 * (f + i);
        acc[0] += p[0];
        acc[1] += p[1];
        acc[2] += p[2];
        acc[3] = fmax(acc[3], p[3]);
    }
    block_sum(acc, out + 4 * c);
}

hipError_t launch_batch_residual(int prec, const void *b0, const void *b1,
                                 const BatchRed *items, int nitems,
                                 const BatchCase *cases, const Geometry *geoms,
                                 const Consts<double> *Kd, const HostSide *H, double *partials,
                                 const int *case_first, const int *case_count, int ncases,
                                 double *out, hipStream_t st) {
    if (nitems > 0) {
        if (f32_storage(prec))
            hipLaunchKernelGGL(batch_residual_kernel<float>, dim3(nitems), dim3(kReduceBlock), 0,
                               st, static_cast<const float *>(b0), static_cast<const float *>(b1),
                               items, cases, geoms, Kd, H, partials);
        else
            hipLaunchKernelGGL(batch_residual_kernel<double>, dim3(nitems), dim3(kReduceBlock), 0,
                               st, static_cast<const double *>(b0), static_cast<const double *>(b1),
                               items, cases, geoms, Kd, H, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(ncases), dim3(kReduceBlock), 0, st, partials,
                       case_first, case_count, out);
    return hipGetLastError();
}

static int reduce_blocks(const Geometry &G) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    long long b = (n + kReduceBlock - 1) / kReduceBlock;
    if (b > kMaxPartials) b = kMaxPartials;
    return static_cast<int>(b);
}

int reduce_partials(const Geometry &G) { return reduce_blocks(G); }

// ------------------------------------------------------------ copy ceiling

// Streaming copy, the reference for what a read-plus-write stream achieves
// on this GPU: 16-byte loads, non-temporal 16-byte stores (the lattice's
// own stores are non-temporal once its buffers exceed the Infinity Cache),
// four independent words per thread per round, grid-stride.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
stream_copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, long long n) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const u32x4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                    d = src[i + 3 * stride];
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(src[i], dst + i);
}

hipError_t launch_stream_copy(void *dst, const void *src, long long n16, int workgroups,
                              hipStream_t st) {
    if (n16 <= 0) return hipSuccess;
    long long g = workgroups > 0 ? workgroups : 8192;
    const long long need = (n16 + 255) / 256;
    if (g > need) g = need;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, st,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

static int conv_blocks(const Geometry &G) {
    const long long n = static_cast<long long>(G.nx) * G.ny;
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return static_cast<int>(b);
}

hipError_t launch_init_feq(int prec, void *dst, const double *rho, const double *ux,
                           const double *uy, const Geometry &G, const HostSide &H,
                           hipStream_t st) {
    if (f32_storage(prec))
        hipLaunchKernelGGL(init_feq_kernel<float>, dim3(conv_blocks(G)), dim3(256), 0, st,
                           static_cast<float *>(dst), rho, ux, uy, G, H);
    else
        hipLaunchKernelGGL(init_feq_kernel<double>, dim3(conv_blocks(G)), dim3(256), 0, st,
                           static_cast<double *>(dst), rho, ux, uy, G, H);
    return hipGetLastError();
}

hipError_t launch_set_populations(int prec, void *dst, const double *f, const Geometry &G,
                                  const HostSide &H, hipStream_t st) {
    if (f32_storage(prec))
        hipLaunchKernelGGL(set_pop_kernel<float>, dim3(conv_blocks(G)), dim3(256), 0, st,
                           static_cast<float *>(dst), f, G, H);
    else
        hipLaunchKernelGGL(set_pop_kernel<double>, dim3(conv_blocks(G)), dim3(256), 0, st,
                           static_cast<double *>(dst), f, G, H);
    return hipGetLastError();
}

hipError_t launch_get_populations(int prec, bool pull, const void *src, double *f,
                                  const Geometry &G, const Consts<double> &Kd,
                                  const Consts<float> &, const HostSide &H, hipStream_t st) {
    const dim3 grid(conv_blocks(G)), block(256);
    if (f32_storage(prec)) {
        const float *s = static_cast<const float *>(src);
        if (pull) hipLaunchKernelGGL((get_pop_kernel<float, true>), grid, block, 0, st, s, f, G, Kd, H);
        else hipLaunchKernelGGL((get_pop_kernel<float, false>), grid, block, 0, st, s, f, G, Kd, H);
    } else {
        const double *s = static_cast<const double *>(src);
        if (pull) hipLaunchKernelGGL((get_pop_kernel<double, true>), grid, block, 0, st, s, f, G, Kd, H);
        else hipLaunchKernelGGL((get_pop_kernel<double, false>), grid, block, 0, st, s, f, G, Kd, H);
    }
    return hipGetLastError();
}

template <typename S>
static void avg_dispatch(bool pc, const S *cur, bool pp, const S *prev, double *f, const Geometry &G,
                         const Consts<double> &Kd, const HostSide &H, hipStream_t st) {
    const dim3 grid(conv_blocks(G)), block(256);
    if (pc && pp) hipLaunchKernelGGL((avg_states_kernel<S, true, true>), grid, block, 0, st, cur, prev, f, G, Kd, H);
    else if (pc) hipLaunchKernelGGL((avg_states_kernel<S, true, false>), grid, block, 0, st, cur, prev, f, G, Kd, H);
    else if (pp) hipLaunchKernelGGL((avg_states_kernel<S, false, true>), grid, block, 0, st, cur, prev, f, G, Kd, H);
    else hipLaunchKernelGGL((avg_states_kernel<S, false, false>), grid, block, 0, st, cur, prev, f, G, Kd, H);
}

hipError_t launch_average_states(int prec, bool pull_cur, const void *cur, bool pull_prev,
                                 const void *prev, double *f, const Geometry &G,
                                 const Consts<double> &Kd, const HostSide &H, hipStream_t st) {
    if (f32_storage(prec))
        avg_dispatch<float>(pull_cur, static_cast<const float *>(cur), pull_prev,
                            static_cast<const float *>(prev), f, G, Kd, H, st);
    else
        avg_dispatch<double>(pull_cur, static_cast<const double *>(cur), pull_prev,
                             static_cast<const double *>(prev), f, G, Kd, H, st);
    return hipGetLastError();
}

hipError_t launch_moments(int prec, bool pull, const void *src, double *rho, double *ux,
                          double *uy, const Geometry &G, const Consts<double> &Kd,
                          const Consts<float> &, const HostSide &H, hipStream_t st) {
    const dim3 grid(conv_blocks(G)), block(256);
    if (f32_storage(prec)) {
        const float *s = static_cast<const float *>(src);
        if (pull) hipLaunchKernelGGL((moments_kernel<float, true>), grid, block, 0, st, s, rho, ux, uy, G, Kd, H);
        else hipLaunchKernelGGL((moments_kernel<float, false>), grid, block, 0, st, s, rho, ux, uy, G, Kd, H);
    } else {
        const double *s = static_cast<const double *>(src);
        if (pull) hipLaunchKernelGGL((moments_kernel<double, true>), grid, block, 0, st, s, rho, ux, uy, G, Kd, H);
        else hipLaunchKernelGGL((moments_kernel<double, false>), grid, block, 0, st, s, rho, ux, uy, G, Kd, H);
    }
    return hipGetLastError();
}

hipError_t launch_stress(int prec, bool pull, const void *src, const double *rho, double *sxx,
                         double *syy, double *sxy, const Geometry &G, const Consts<double> &Kd,
                         const HostSide &H, hipStream_t st) {
    const dim3 grid(conv_blocks(G)), block(256);
    if (f32_storage(prec)) {
        const float *s = static_cast<const float *>(src);
        if (pull) hipLaunchKernelGGL((stress_kernel<float, true>), grid, block, 0, st, s, rho, sxx, syy, sxy, G, Kd, H);
        else hipLaunchKernelGGL((stress_kernel<float, false>), grid, block, 0, st, s, rho, sxx, syy, sxy, G, Kd, H);
    } else {
        const double *s = static_cast<const double *>(src);
        if (pull) hipLaunchKernelGGL((stress_kernel<double, true>), grid, block, 0, st, s, rho, sxx, syy, sxy, G, Kd, H);
        else hipLaunchKernelGGL((stress_kernel<double, false>), grid, block, 0, st, s, rho, sxx, syy, sxy, G, Kd, H);
    }
    return hipGetLastError();
}

hipError_t launch_sums(int prec, bool pull, const void *src, double *partials, double *out,
                       const Geometry &G, const Consts<double> &Kd, const Consts<float> &,
                       const HostSide &H, hipStream_t st) {
    const int nb = reduce_blocks(G);
    const dim3 grid(nb), block(kReduceBlock);
    if (f32_storage(prec)) {
        const float *s = static_cast<const float *>(src);
        if (pull) hipLaunchKernelGGL((sums_kernel<float, true>), grid, block, 0, st, s, partials, G, Kd, H);
        else hipLaunchKernelGGL((sums_kernel<float, false>), grid, block, 0, st, s, partials, G, Kd, H);
    } else {
        const double *s = static_cast<const double *>(src);
        if (pull) hipLaunchKernelGGL((sums_kernel<double, true>), grid, block, 0, st, s, partials, G, Kd, H);
        else hipLaunchKernelGGL((sums_kernel<double, false>), grid, block, 0, st, s, partials, G, Kd, H);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<4>, dim3(1), dim3(kReduceBlock), 0, st, partials, nb, out);
    return hipGetLastError();
}

template <typename S>
static void residual_dispatch(bool pc, const S *cur, bool pp, const S *prev, double *partials,
                              const Geometry &G, const Consts<double> &Kd, const HostSide &H,
                              int nb, hipStream_t st) {
    const dim3 grid(nb), block(kReduceBlock);
    if (pc && pp) hipLaunchKernelGGL((residual_kernel<S, S, true, true>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else if (pc) hipLaunchKernelGGL((residual_kernel<S, S, true, false>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else if (pp) hipLaunchKernelGGL((residual_kernel<S, S, false, true>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else hipLaunchKernelGGL((residual_kernel<S, S, false, false>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
}

hipError_t launch_residual(int prec, bool pull_cur, const void *cur, bool pull_prev,
                           const void *prev, double *partials, double *out, const Geometry &G,
                           const Consts<double> &Kd, const Consts<float> &, const HostSide &H,
                           hipStream_t st) {
    const int nb = reduce_blocks(G);
    if (f32_storage(prec))
        residual_dispatch<float>(pull_cur, static_cast<const float *>(cur), pull_prev,
                                 static_cast<const float *>(prev), partials, G, Kd, H, nb, st);
    else
        residual_dispatch<double>(pull_cur, static_cast<const double *>(cur), pull_prev,
                                  static_cast<const double *>(prev), partials, G, Kd, H, nb, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<4>, dim3(1), dim3(kReduceBlock), 0, st, partials, nb, out);
    return hipGetLastError();
}

template <typename S>
static void check_dispatch(bool pc, const S *cur, bool pp, const S *prev, double *partials,
                           const Geometry &G, const Consts<double> &Kd, const HostSide &H, int nb,
                           hipStream_t st) {
    const dim3 grid(nb), block(kReduceBlock);
    if (pc && pp) hipLaunchKernelGGL((check_kernel<S, true, true>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else if (pc) hipLaunchKernelGGL((check_kernel<S, true, false>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else if (pp) hipLaunchKernelGGL((check_kernel<S, false, true>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
    else hipLaunchKernelGGL((check_kernel<S, false, false>), grid, block, 0, st, cur, prev, partials, G, Kd, H);
}

hipError_t launch_check(int prec, bool pull_cur, const void *cur, bool pull_prev,
                        const void *prev, double *partials, double *out, const Geometry &G,
                        const Consts<double> &Kd, const Consts<float> &, const HostSide &H,
                        hipStream_t st) {
    const int nb = reduce_blocks(G);
    if (f32_storage(prec))
        check_dispatch<float>(pull_cur, static_cast<const float *>(cur), pull_prev,
                              static_cast<const float *>(prev), partials, G, Kd, H, nb, st);
    else
        check_dispatch<double>(pull_cur, static_cast<const double *>(cur), pull_prev,
                               static_cast<const double *>(prev), partials, G, Kd, H, nb, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<8>, dim3(1), dim3(kReduceBlock), 0, st, partials, nb, out);
    return hipGetLastError();
}

}  // namespace lbm
