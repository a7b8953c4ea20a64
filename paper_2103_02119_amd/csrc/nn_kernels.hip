// Kernels of the learned warm start: a convolutional encoder-decoder whose
// 3x3 convolutions run as implicit GEMMs on the CDNA matrix cores in BF16
// with FP32 accumulation, plus the elementwise pieces of its forward and
// backward passes and the optimizer.  Declared in include/lbm_nn.h.
//
// Tensors are NHWC.  Forward activations are BF16; gradients are FP32 (they
// are rounded to BF16 only as matrix-core operands).  A 3x3 weight is stored
// as W[k][co] with k = tap * C + ci, tap = 3 (dy + 1) + (dx + 1): the output
// at pixel (y, x) reads the input at (y + dy, x + dx), zero outside.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdk = kBK + 8;  // padded LDS row (bf16 elements) of the k-contiguous tiles
constexpr int kThreads = 256;  // 4 wavefronts, 2 x 2 over the 64 x 64 output tile

// v_mfma_f32_16x16x32_bf16 operand layout (lane l, element e):
//   A[i][k]: i = l % 16, k = 8 (l / 16) + e;  B[k][j]: j = l % 16, k = 8 (l / 16) + e;
//   D[i][j]: j = l % 16, i = 4 (l / 16) + e.
// Each wavefront owns a 32 x 32 block of the tile: 2 x 2 of these products per
// 32-deep slice of k, read from k-contiguous LDS rows (16 bytes per lane).
__device__ __forceinline__ void mma_slice(const bf16 (*As)[kLdk], const bf16 (*Bt)[kLdk],
                                          int wm, int wn, int lane, f32x4 (&acc)[2][2]) {
    const int r = lane & 15, kk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + r][kk]);
        b[i] = *reinterpret_cast<const bf16x8 *>(&Bt[wn * 32 + i * 16 + r][kk]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
}

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 load8_f32(const float *p) {
    const float4 u = *reinterpret_cast<const float4 *>(p);
    const float4 v = *reinterpret_cast<const float4 *>(p + 4);
    bf16x8 r;
    r[0] = (bf16)u.x; r[1] = (bf16)u.y; r[2] = (bf16)u.z; r[3] = (bf16)u.w;
    r[4] = (bf16)v.x; r[5] = (bf16)v.y; r[6] = (bf16)v.z; r[7] = (bf16)v.w;
    return r;
}

// ---------------------------------------------------------------- 3x3 forward
// Y[m][co] = act(sum_k X(m, k) W[k][co] + b[co]); X is the channel concat of
// x1 (c1 channels) and x2 (c2), k = tap (c1 + c2) + ci.  wt is W transposed
// (WT[co][k], k contiguous) in BF16.
__global__ void __launch_bounds__(kThreads)
conv_fwd_kernel(const bf16 *__restrict__ x1, int c1, const bf16 *__restrict__ x2, int c2, int N,
                int H, int W, const bf16 *__restrict__ wt, const float *__restrict__ bias,
                int cout, int relu, bf16 *__restrict__ y) {
    __shared__ __attribute__((aligned(16))) bf16 As[kBM][kLdk];
    __shared__ __attribute__((aligned(16))) bf16 Bt[kBN][kLdk];
    const int C = c1 + c2, K = 9 * C, M = N * H * W;
    const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int ar = t >> 2, kc = (t & 3) * 8;
    const int m = m0 + ar;
    const int pn = m / (H * W), py = (m / W) % H, px = m % W;
    const int n = n0 + ar;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const int k = k0 + kc;  // 8 consecutive k share a tap (C % 8 == 0)
        bf16x8 av = zero8(), bv = zero8();
        if (m < M && k < K) {
            const int tap = k / C, ci = k - tap * C;
            const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
                const size_t pix = (static_cast<size_t>(pn) * H + yy) * W + xx;
                av = ci < c1 ? *reinterpret_cast<const bf16x8 *>(x1 + pix * c1 + ci)
                             : *reinterpret_cast<const bf16x8 *>(x2 + pix * c2 + (ci - c1));
            }
        }
        if (n < cout && k < K) bv = *reinterpret_cast<const bf16x8 *>(wt + static_cast<size_t>(n) * K + k);
        *reinterpret_cast<bf16x8 *>(&As[ar][kc]) = av;
        *reinterpret_cast<bf16x8 *>(&Bt[ar][kc]) = bv;
        __syncthreads();
        mma_slice(As, Bt, wm, wn, lane, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int mm = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (mm < M && nn < cout) {
                    float v = acc[i][j][e] + bias[nn];
                    if (relu) v = v > 0.f ? v : 0.f;
                    y[static_cast<size_t>(mm) * cout + nn] = (bf16)v;
                }
            }
}

// ---------------------------------------------------------------- 3x3 data gradient
// gX(p, ci) = sum_{tap, co} gY(p - off(tap), co) W[tap C + ci][co]: a GEMM over
// k' = tap cout + co with B[k'][ci] = W[tap C + ci][co] held as WD[ci][k']
// (k' contiguous) in BF16.  The result is split over the concat inputs and
// written or added (accumulate) in FP32.
__global__ void __launch_bounds__(kThreads)
conv_dgrad_kernel(const float *__restrict__ gy, int N, int H, int W, int cout,
                  const bf16 *__restrict__ wd, float *__restrict__ gx1, int c1,
                  float *__restrict__ gx2, int c2, int accumulate) {
    __shared__ __attribute__((aligned(16))) bf16 As[kBM][kLdk];
    __shared__ __attribute__((aligned(16))) bf16 Bt[kBN][kLdk];
    const int C = c1 + c2, K = 9 * cout, M = N * H * W;
    const int m0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int ar = t >> 2, kc = (t & 3) * 8;
    const int m = m0 + ar;
    const int pn = m / (H * W), py = (m / W) % H, px = m % W;
    const int n = n0 + ar;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kBK) {
        const int k = k0 + kc;  // 8 consecutive k share a tap (cout % 8 == 0)
        bf16x8 av = zero8(), bv = zero8();
        if (m < M && k < K) {
            const int tap = k / cout, co = k - tap * cout;
            const int yy = py - (tap / 3 - 1), xx = px - (tap % 3 - 1);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                av = load8_f32(gy + ((static_cast<size_t>(pn) * H + yy) * W + xx) * cout + co);
        }
        if (n < C && k < K) bv = *reinterpret_cast<const bf16x8 *>(wd + static_cast<size_t>(n) * K + k);
        *reinterpret_cast<bf16x8 *>(&As[ar][kc]) = av;
        *reinterpret_cast<bf16x8 *>(&Bt[ar][kc]) = bv;
        __syncthreads();
        mma_slice(As, Bt, wm, wn, lane, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int mm = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (mm < M && nn < C) {
                    float *dst = nn < c1 ? gx1 + static_cast<size_t>(mm) * c1 + nn
                                         : gx2 + static_cast<size_t>(mm) * c2 + (nn - c1);
                    const float v = acc[i][j][e];
                    *dst = accumulate ? *dst + v : v;
                }
            }
}

// ---------------------------------------------------------------- 3x3 weight gradient
// part[s][k][co] = sum over the pixels of split s of X(m, k) gY(m, co): A is
// X^T (rows k, pixels along the reduction) and B is gY, both staged through
// LDS transposed so that each lane reads 8 consecutive pixels.
__global__ void __launch_bounds__(kThreads)
conv_wgrad_kernel(const bf16 *__restrict__ x1, int c1, const bf16 *__restrict__ x2, int c2,
                  int N, int H, int W, const float *__restrict__ gy, int cout, int chunk,
                  float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16 As[kBM][kLdk];  // [k][pixel]
    __shared__ __attribute__((aligned(16))) bf16 Bt[kBN][kLdk];  // [co][pixel]
    const int C = c1 + c2, K = 9 * C, M = N * H * W;
    const int k0 = blockIdx.x * kBM, n0 = blockIdx.y * kBN, s = blockIdx.z;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wm = wv >> 1, wn = wv & 1;
    const int pm = t >> 3, cc = (t & 7) * 8;  // this thread's pixel row and 8-wide chunk
    const int mbeg = s * chunk, mend = min(M, mbeg + chunk);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int k = k0 + cc;
    const int tap = k < K ? k / C : 0, ci = k - tap * C;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int co = n0 + cc;
    for (int p0 = mbeg; p0 < mend; p0 += kBK) {
        const int m = p0 + pm;
        bf16x8 av = zero8(), bv = zero8();
        if (m < mend) {
            const int pn = m / (H * W), py = (m / W) % H, px = m % W;
            const int yy = py + dy, xx = px + dx;
            if (k < K && yy >= 0 && yy < H && xx >= 0 && xx < W) {
                const size_t pix = (static_cast<size_t>(pn) * H + yy) * W + xx;
                av = ci < c1 ? *reinterpret_cast<const bf16x8 *>(x1 + pix * c1 + ci)
                             : *reinterpret_cast<const bf16x8 *>(x2 + pix * c2 + (ci - c1));
            }
            if (co < cout) bv = load8_f32(gy + static_cast<size_t>(m) * cout + co);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            As[cc + e][pm] = av[e];
            Bt[cc + e][pm] = bv[e];
        }
        __syncthreads();
        mma_slice(As, Bt, wm, wn, lane, acc);
        __syncthreads();
    }
    float *out = part + static_cast<size_t>(s) * K * cout;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int kk = k0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (kk < K && nn < cout) out[static_cast<size_t>(kk) * cout + nn] = acc[i][j][e];
            }
}

// gw[i] = sum_s part[s][i] in a fixed order: a block takes kSumOuts
// consecutive outputs, its kSumGroups thread groups each sum every
// kSumGroups-th split (s = group, group + kSumGroups, ...), and the group
// sums are added in group order.
constexpr int kSumOuts = 32, kSumGroups = 8;
__global__ void __launch_bounds__(kSumOuts * kSumGroups)
sum_splits_kernel(const float *__restrict__ part, int splits, size_t n, float *__restrict__ gw) {
    __shared__ float red[kSumGroups][kSumOuts];
    const int lo = static_cast<int>(threadIdx.x) % kSumOuts;
    const int grp = static_cast<int>(threadIdx.x) / kSumOuts;
    for (size_t base = static_cast<size_t>(blockIdx.x) * kSumOuts; base < n;
         base += static_cast<size_t>(gridDim.x) * kSumOuts) {
        const size_t i = base + lo;
        float s = 0.f;
        if (i < n)
            for (int j = grp; j < splits; j += kSumGroups) s += part[static_cast<size_t>(j) * n + i];
        red[grp][lo] = s;
        __syncthreads();
        if (grp == 0 && i < n) {
            float t = 0.f;
            for (int q = 0; q < kSumGroups; ++q) t += red[q][lo];
            gw[i] = t;
        }
        __syncthreads();  // red is reused by the next outputs
    }
}

int sum_grid(size_t n) {
    size_t b = (n + kSumOuts - 1) / kSumOuts;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : static_cast<int>(b);
}

// per-block column sums of g[M][c] (block b covers rows b*rows .. ), then a
// fixed-order sum over blocks.  Within a block the threads form groups of W
// columns (W = c, or the block width for wider rows); group q sums rows
// r0 + q, r0 + q + G, ... and the G group sums are added in group order.
constexpr int kColThreads = 256;
__global__ void __launch_bounds__(kColThreads)
colsum_partial_kernel(const float *__restrict__ g, int M, int c, int rows,
                      float *__restrict__ part) {
    __shared__ float red[kColThreads];
    const int r0 = blockIdx.x * rows, r1 = min(M, r0 + rows);
    const int W = c < kColThreads ? c : kColThreads;
    const int G = kColThreads / W;
    const int t = static_cast<int>(threadIdx.x), grp = t / W, jl = t % W;
    for (int j0 = 0; j0 < c; j0 += W) {
        const int j = j0 + jl;
        float s = 0.f;
        if (grp < G && j < c)
            for (int r = r0 + grp; r < r1; r += G) s += g[static_cast<size_t>(r) * c + j];
        red[t] = s;
        __syncthreads();
        if (grp == 0 && j < c) {
            float tot = 0.f;
            for (int q = 0; q < G; ++q) tot += red[q * W + jl];
            part[static_cast<size_t>(blockIdx.x) * c + j] = tot;
        }
        __syncthreads();  // red is reused by the next columns
    }
}

// ---------------------------------------------------------------- elementwise
__global__ void relu_bwd_kernel(const float *__restrict__ gy, const bf16 *__restrict__ y,
                                float *__restrict__ g, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        g[i] = static_cast<float>(y[i]) > 0.f ? gy[i] : 0.f;
}

// The pooling and upsampling kernels take the index type I: 32-bit unsigned
// when every buffer they touch has fewer than 2^32 elements (the division
// and modulo of the index then run in 32 bits), size_t otherwise.

// 2 x 2 average pooling, x [N][H][W][c] -> y [N][H/2][W/2][c]
template <typename I>
__global__ void avgpool_fwd_kernel(const bf16 *__restrict__ x, int N, int H, int W, int c,
                                   bf16 *__restrict__ y) {
    const I Ho = H / 2, Wo = W / 2, C = c, Wi = W, Hi = H;
    const I n = static_cast<I>(N) * Ho * Wo * C;
    for (I i = blockIdx.x * static_cast<I>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<I>(gridDim.x) * blockDim.x) {
        const I ch = i % C;
        const I p = i / C;
        const I xo = p % Wo, yo = (p / Wo) % Ho;
        const I b = p / (Wo * Ho);
        const I base = ((b * Hi + 2 * yo) * Wi + 2 * xo) * C + ch;
        const float s = static_cast<float>(x[base]) + static_cast<float>(x[base + C]) +
                        static_cast<float>(x[base + Wi * C]) +
                        static_cast<float>(x[base + Wi * C + C]);
        y[i] = (bf16)(0.25f * s);
    }
}

// gx [N][H][W][c] (+)= gy [N][H/2][W/2][c] / 4 on each of the 2 x 2 sources
template <typename I>
__global__ void avgpool_bwd_kernel(const float *__restrict__ gy, int N, int H, int W, int c,
                                   float *__restrict__ gx, int accumulate) {
    const I Hi = H, Wi = W, C = c, Ho = H / 2, Wo = W / 2;
    const I n = static_cast<I>(N) * Hi * Wi * C;
    for (I i = blockIdx.x * static_cast<I>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<I>(gridDim.x) * blockDim.x) {
        const I ch = i % C;
        const I p = i / C;
        const I xx = p % Wi, yy = (p / Wi) % Hi;
        const I b = p / (Wi * Hi);
        const float v = 0.25f * gy[((b * Ho + yy / 2) * Wo + xx / 2) * C + ch];
        gx[i] = accumulate ? gx[i] + v : v;
    }
}

// nearest upsampling by 2, x [N][H][W][c] -> y [N][2H][2W][c]
template <typename I>
__global__ void upsample_fwd_kernel(const bf16 *__restrict__ x, int N, int H, int W, int c,
                                    bf16 *__restrict__ y) {
    const I Hi = H, Wi = W, C = c, Ho = 2 * Hi, Wo = 2 * Wi;
    const I n = static_cast<I>(N) * Ho * Wo * C;
    for (I i = blockIdx.x * static_cast<I>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<I>(gridDim.x) * blockDim.x) {
        const I ch = i % C;
        const I p = i / C;
        const I xo = p % Wo, yo = (p / Wo) % Ho;
        const I b = p / (Wo * Ho);
        y[i] = x[((b * Hi + yo / 2) * Wi + xo / 2) * C + ch];
    }
}

// gx [N][H][W][c] = sum of gy over the 2 x 2 copies
template <typename I>
__global__ void upsample_bwd_kernel(const float *__restrict__ gy, int N, int H, int W, int c,
                                    float *__restrict__ gx) {
    const I Hi = H, Wi = W, C = c, Wo = 2 * Wi;
    const I n = static_cast<I>(N) * Hi * Wi * C;
    for (I i = blockIdx.x * static_cast<I>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<I>(gridDim.x) * blockDim.x) {
        const I ch = i % C;
        const I p = i / C;
        const I xx = p % Wi, yy = (p / Wi) % Hi;
        const I b = p / (Wi * Hi);
        const I q = ((b * 2 * Hi + 2 * yy) * Wo + 2 * xx) * C + ch;
        gx[i] = (gy[q] + gy[q + C]) + (gy[q + Wo * C] + gy[q + Wo * C + C]);
    }
}

// true when buffers of `elems` elements can be indexed in 32 bits, with
// room for one more grid stride (grid_for: at most 65536 x 256 threads)
bool fits32(size_t elems) {
    return elems + (static_cast<size_t>(1) << 24) < (static_cast<size_t>(1) << 32);
}

// 1x1 head: y[m][o] = sum_i x[m][i] w[i][o] + b[o] (FP32 out)
__global__ void conv1x1_fwd_kernel(const bf16 *__restrict__ x, int M, int cin,
                                   const float *__restrict__ w, const float *__restrict__ b,
                                   int cout, float *__restrict__ y) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
         i < static_cast<size_t>(M) * cout; i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t m = i / cout;
        const int o = static_cast<int>(i % cout);
        float s = b[o];
        for (int j = 0; j < cin; ++j) s += static_cast<float>(x[m * cin + j]) * w[j * cout + o];
        y[i] = s;
    }
}

// gx[m][i] = sum_o gy[m][o] w[i][o]
__global__ void conv1x1_dgrad_kernel(const float *__restrict__ gy, int M, int cin,
                                     const float *__restrict__ w, int cout,
                                     float *__restrict__ gx) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
         i < static_cast<size_t>(M) * cin; i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t m = i / cin;
        const int j = static_cast<int>(i % cin);
        float s = 0.f;
        for (int o = 0; o < cout; ++o) s += gy[m * cout + o] * w[j * cout + o];
        gx[i] = s;
    }
}

// part[b][i][o] = sum over rows of block b of x[m][i] gy[m][o]
__global__ void conv1x1_wgrad_partial_kernel(const bf16 *__restrict__ x, const float *__restrict__ gy,
                                             int M, int cin, int cout, int rows,
                                             float *__restrict__ part) {
    const int r0 = blockIdx.x * rows, r1 = min(M, r0 + rows);
    for (int q = threadIdx.x; q < cin * cout; q += blockDim.x) {
        const int j = q / cout, o = q % cout;
        float s = 0.f;
        for (int r = r0; r < r1; ++r)
            s += static_cast<float>(x[static_cast<size_t>(r) * cin + j]) * gy[static_cast<size_t>(r) * cout + o];
        part[static_cast<size_t>(blockIdx.x) * cin * cout + q] = s;
    }
}

// masked mean-square error: per pixel weight fluid[m] (0 / 1), per channel
// weight cw[c]; part[b] = this block's sum, grad = d loss / d pred
__global__ void mse_kernel(const float *__restrict__ pred, const float *__restrict__ tgt,
                           const unsigned char *__restrict__ fluid, int M, int c,
                           const float *__restrict__ cw, float inv_count,
                           float *__restrict__ grad, float *__restrict__ part) {
    __shared__ float red[kThreads];
    float s = 0.f;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
         i < static_cast<size_t>(M) * c; i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t m = i / c;
        const int ch = static_cast<int>(i % c);
        const float w = fluid[m] ? cw[ch] : 0.f;
        const float d = pred[i] - tgt[i];
        s += w * d * d;
        grad[i] = 2.f * w * d * inv_count;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv_count;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, size_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// W[k = tap C + ci][co] (FP32) -> WT[co][k] and WD[ci][tap cout + co] (BF16)
__global__ void cast_weights_kernel(const float *__restrict__ w, int C, int cout,
                                    bf16 *__restrict__ wt, bf16 *__restrict__ wd) {
    const size_t n = static_cast<size_t>(9) * C * cout;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int co = static_cast<int>(i % cout);
        const size_t k = i / cout;
        const int tap = static_cast<int>(k / C), ci = static_cast<int>(k % C);
        const bf16 b = (bf16)w[i];
        wt[static_cast<size_t>(co) * 9 * C + k] = b;
        wd[static_cast<size_t>(ci) * 9 * cout + static_cast<size_t>(tap) * cout + co] = b;
    }
}

__global__ void cast_bf16_kernel(const float *__restrict__ x, size_t n, bf16 *__restrict__ y) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        y[i] = (bf16)x[i];
}

int grid_for(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : static_cast<int>(b);
}

int check(hipError_t e) { return e == hipSuccess ? LBM_NN_OK : LBM_NN_E_DEVICE; }

}  // namespace

extern "C" {

int lbm_nn_conv3x3_fwd(const void *x1, int c1, const void *x2, int c2, int n, int h, int w,
                       const void *wt, const float *bias, int cout, int relu, void *y,
                       void *stream) {
    if (!x1 || !wt || !bias || !y || n < 1 || h < 1 || w < 1 || c1 < 8 || c1 % 8 || c2 < 0 ||
        c2 % 8 || (c2 > 0 && !x2) || cout < 1)
        return LBM_NN_E_INVAL;
    const long long M = static_cast<long long>(n) * h * w;
    if (M > 0x7fffffffLL) return LBM_NN_E_INVAL;
    const dim3 grid(static_cast<unsigned>((M + kBM - 1) / kBM), (cout + kBN - 1) / kBN);
    hipLaunchKernelGGL(conv_fwd_kernel, grid, dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16 *>(x1), c1, static_cast<const bf16 *>(x2), c2, n, h,
                       w, static_cast<const bf16 *>(wt), bias, cout, relu, static_cast<bf16 *>(y));
    return check(hipGetLastError());
}

int lbm_nn_conv3x3_dgrad(const float *gy, int n, int h, int w, int cout, const void *wd,
                         float *gx1, int c1, float *gx2, int c2, int accumulate, void *stream) {
    if (!gy || !wd || !gx1 || n < 1 || h < 1 || w < 1 || cout < 8 || cout % 8 || c1 < 1 ||
        c2 < 0 || (c2 > 0 && !gx2))
        return LBM_NN_E_INVAL;
    const long long M = static_cast<long long>(n) * h * w;
    if (M > 0x7fffffffLL) return LBM_NN_E_INVAL;
    const dim3 grid(static_cast<unsigned>((M + kBM - 1) / kBM), (c1 + c2 + kBN - 1) / kBN);
    hipLaunchKernelGGL(conv_dgrad_kernel, grid, dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), gy, n, h, w, cout,
                       static_cast<const bf16 *>(wd), gx1, c1, gx2, c2, accumulate);
    return check(hipGetLastError());
}

size_t lbm_nn_conv3x3_wgrad_work(int c1, int c2, int n, int h, int w, int cout) {
    const long long M = static_cast<long long>(n) * h * w;
    const int C = c1 + c2, K = 9 * C;
    const long long tiles = static_cast<long long>((K + kBM - 1) / kBM) * ((cout + kBN - 1) / kBN);
    long long splits = (1024 + tiles - 1) / tiles;
    const long long maxs = (M + 4 * kBK - 1) / (4 * kBK);
    if (splits > maxs) splits = maxs;
    if (splits < 1) splits = 1;
    const long long cols_parts = (M + 511) / 512;
    const size_t a = static_cast<size_t>(splits) * K * cout * sizeof(float);
    const size_t b = static_cast<size_t>(cols_parts) * cout * sizeof(float);
    return a > b ? a : b;
}

int lbm_nn_conv3x3_wgrad(const void *x1, int c1, const void *x2, int c2, int n, int h, int w,
                         const float *gy, int cout, float *gw, float *gb, void *work,
                         size_t work_bytes, void *stream) {
    if (!x1 || !gy || !gw || !gb || !work || n < 1 || h < 1 || w < 1 || c1 < 8 || c1 % 8 ||
        c2 < 0 || c2 % 8 || (c2 > 0 && !x2) || cout < 8 || cout % 8)
        return LBM_NN_E_INVAL;
    if (work_bytes < lbm_nn_conv3x3_wgrad_work(c1, c2, n, h, w, cout)) return LBM_NN_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long M = static_cast<long long>(n) * h * w;
    const int C = c1 + c2, K = 9 * C;
    const long long tiles = static_cast<long long>((K + kBM - 1) / kBM) * ((cout + kBN - 1) / kBN);
    long long splits = (1024 + tiles - 1) / tiles;
    const long long maxs = (M + 4 * kBK - 1) / (4 * kBK);
    if (splits > maxs) splits = maxs;
    if (splits < 1) splits = 1;
    long long chunk = (M + splits - 1) / splits;
    chunk = (chunk + kBK - 1) / kBK * kBK;
    splits = (M + chunk - 1) / chunk;
    float *part = static_cast<float *>(work);
    const dim3 grid((K + kBM - 1) / kBM, (cout + kBN - 1) / kBN, static_cast<unsigned>(splits));
    hipLaunchKernelGGL(conv_wgrad_kernel, grid, dim3(kThreads), 0, st,
                       static_cast<const bf16 *>(x1), c1, static_cast<const bf16 *>(x2), c2, n, h,
                       w, gy, cout, static_cast<int>(chunk), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return LBM_NN_E_DEVICE;
    const size_t nw = static_cast<size_t>(K) * cout;
    hipLaunchKernelGGL(sum_splits_kernel, dim3(sum_grid(nw)), dim3(kSumOuts * kSumGroups), 0, st,
                       part, static_cast<int>(splits), nw, gw);
    // bias gradient: column sums of gy, reusing the work space after the sum
    const int rows = 512;
    const int nb = static_cast<int>((M + rows - 1) / rows);
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(nb), dim3(kColThreads), 0, st, gy,
                       static_cast<int>(M), cout, rows, part);
    hipLaunchKernelGGL(sum_splits_kernel, dim3(sum_grid(cout)), dim3(kSumOuts * kSumGroups), 0,
                       st, part, nb, static_cast<size_t>(cout), gb);
    return check(hipGetLastError());
}

int lbm_nn_relu_bwd(const float *gy, const void *y, float *g, size_t count, void *stream) {
    if (!gy || !y || !g) return LBM_NN_E_INVAL;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid_for(count)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), gy, static_cast<const bf16 *>(y), g, count);
    return check(hipGetLastError());
}

int lbm_nn_avgpool2_fwd(const void *x, int n, int h, int w, int c, void *y, void *stream) {
    if (!x || !y || n < 1 || h < 2 || w < 2 || (h & 1) || (w & 1) || c < 1) return LBM_NN_E_INVAL;
    const size_t cnt = static_cast<size_t>(n) * (h / 2) * (w / 2) * c;
    const auto *xp = static_cast<const bf16 *>(x);
    auto *yp = static_cast<bf16 *>(y);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fits32(4 * cnt))
        hipLaunchKernelGGL(avgpool_fwd_kernel<uint32_t>, dim3(grid_for(cnt)), dim3(256), 0, st, xp,
                           n, h, w, c, yp);
    else
        hipLaunchKernelGGL(avgpool_fwd_kernel<size_t>, dim3(grid_for(cnt)), dim3(256), 0, st, xp,
                           n, h, w, c, yp);
    return check(hipGetLastError());
}

int lbm_nn_avgpool2_bwd(const float *gy, int n, int h, int w, int c, float *gx, int accumulate,
                        void *stream) {
    if (!gy || !gx || n < 1 || h < 2 || w < 2 || (h & 1) || (w & 1) || c < 1) return LBM_NN_E_INVAL;
    const size_t cnt = static_cast<size_t>(n) * h * w * c;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fits32(cnt))
        hipLaunchKernelGGL(avgpool_bwd_kernel<uint32_t>, dim3(grid_for(cnt)), dim3(256), 0, st, gy,
                           n, h, w, c, gx, accumulate);
    else
        hipLaunchKernelGGL(avgpool_bwd_kernel<size_t>, dim3(grid_for(cnt)), dim3(256), 0, st, gy,
                           n, h, w, c, gx, accumulate);
    return check(hipGetLastError());
}

int lbm_nn_upsample2_fwd(const void *x, int n, int h, int w, int c, void *y, void *stream) {
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return LBM_NN_E_INVAL;
    const size_t cnt = static_cast<size_t>(n) * 4 * h * w * c;
    const auto *xp = static_cast<const bf16 *>(x);
    auto *yp = static_cast<bf16 *>(y);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fits32(cnt))
        hipLaunchKernelGGL(upsample_fwd_kernel<uint32_t>, dim3(grid_for(cnt)), dim3(256), 0, st, xp,
                           n, h, w, c, yp);
    else
        hipLaunchKernelGGL(upsample_fwd_kernel<size_t>, dim3(grid_for(cnt)), dim3(256), 0, st, xp,
                           n, h, w, c, yp);
    return check(hipGetLastError());
}

int lbm_nn_upsample2_bwd(const float *gy, int n, int h, int w, int c, float *gx, void *stream) {
    if (!gy || !gx || n < 1 || h < 1 || w < 1 || c < 1) return LBM_NN_E_INVAL;
    const size_t cnt = static_cast<size_t>(n) * h * w * c;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (fits32(4 * cnt))
        hipLaunchKernelGGL(upsample_bwd_kernel<uint32_t>, dim3(grid_for(cnt)), dim3(256), 0, st, gy,
                           n, h, w, c, gx);
    else
        hipLaunchKernelGGL(upsample_bwd_kernel<size_t>, dim3(grid_for(cnt)), dim3(256), 0, st, gy,
                           n, h, w, c, gx);
    return check(hipGetLastError());
}

int lbm_nn_conv1x1_fwd(const void *x, int m, int cin, const float *w, const float *b, int cout,
                       float *y, void *stream) {
    if (!x || !w || !b || !y || m < 1 || cin < 1 || cout < 1) return LBM_NN_E_INVAL;
    hipLaunchKernelGGL(conv1x1_fwd_kernel, dim3(grid_for(static_cast<size_t>(m) * cout)), dim3(256),
                       0, static_cast<hipStream_t>(stream), static_cast<const bf16 *>(x), m, cin, w,
                       b, cout, y);
    return check(hipGetLastError());
}

size_t lbm_nn_conv1x1_work(int m, int cin, int cout) {
    const size_t nb = (static_cast<size_t>(m) + 1023) / 1024;
    const size_t a = nb * cin * cout, b = nb * cout;
    return (a > b ? a : b) * sizeof(float);
}

int lbm_nn_conv1x1_bwd(const void *x, const float *gy, int m, int cin, const float *w, int cout,
                       float *gx, float *gw, float *gb, void *work, size_t work_bytes,
                       void *stream) {
    if (!x || !gy || !w || !gx || !gw || !gb || !work || m < 1 || cin < 1 || cout < 1)
        return LBM_NN_E_INVAL;
    if (work_bytes < lbm_nn_conv1x1_work(m, cin, cout)) return LBM_NN_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(conv1x1_dgrad_kernel, dim3(grid_for(static_cast<size_t>(m) * cin)),
                       dim3(256), 0, st, gy, m, cin, w, cout, gx);
    const int rows = 1024, nb = (m + rows - 1) / rows;
    float *part = static_cast<float *>(work);
    hipLaunchKernelGGL(conv1x1_wgrad_partial_kernel, dim3(nb), dim3(256), 0, st,
                       static_cast<const bf16 *>(x), gy, m, cin, cout, rows, part);
    const size_t nw = static_cast<size_t>(cin) * cout;
    hipLaunchKernelGGL(sum_splits_kernel, dim3(sum_grid(nw)), dim3(kSumOuts * kSumGroups), 0, st,
                       part, nb, nw, gw);
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(nb), dim3(kColThreads), 0, st, gy, m, cout,
                       rows, part);
    hipLaunchKernelGGL(sum_splits_kernel, dim3(sum_grid(cout)), dim3(kSumOuts * kSumGroups), 0,
                       st, part, nb, static_cast<size_t>(cout), gb);
    return check(hipGetLastError());
}

size_t lbm_nn_mse_work(int m, int c) {
    const size_t n = static_cast<size_t>(m) * c;
    size_t b = (n + 255) / 256;
    if (b > 1024) b = 1024;
    return (b + 1) * sizeof(float);
}

int lbm_nn_mse(const float *pred, const float *target, const unsigned char *fluid, int m, int c,
               const float *cw, float count, float *grad, float *loss, void *work,
               size_t work_bytes, void *stream) {
    if (!pred || !target || !fluid || !cw || !grad || !loss || !work || m < 1 || c < 1 ||
        !(count > 0.f))
        return LBM_NN_E_INVAL;
    if (work_bytes < lbm_nn_mse_work(m, c)) return LBM_NN_E_INVAL;
    const size_t n = static_cast<size_t>(m) * c;
    int nb = static_cast<int>((n + 255) / 256);
    if (nb > 1024) nb = 1024;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *part = static_cast<float *>(work);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(kThreads), 0, st, pred, target, fluid, m, c, cw,
                       1.f / count, grad, part);
    hipLaunchKernelGGL(sum_splits_kernel, dim3(1), dim3(kSumOuts * kSumGroups), 0, st, part, nb,
                       static_cast<size_t>(1),
                       loss);
    return check(hipGetLastError());
}

int lbm_nn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                float b2, float eps, int step, void *stream) {
    if (!p || !g || !m || !v || step < 1) return LBM_NN_E_INVAL;
    const float c1 = 1.f / (1.f - powf(b1, static_cast<float>(step)));
    const float c2 = 1.f / (1.f - powf(b2, static_cast<float>(step)));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return check(hipGetLastError());
}

int lbm_nn_cast_weights(const float *w, int c, int cout, void *wt, void *wd, void *stream) {
    if (!w || !wt || !wd || c < 1 || cout < 1) return LBM_NN_E_INVAL;
    const size_t n = static_cast<size_t>(9) * c * cout;
    hipLaunchKernelGGL(cast_weights_kernel, dim3(grid_for(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), w, c, cout, static_cast<bf16 *>(wt),
                       static_cast<bf16 *>(wd));
    return check(hipGetLastError());
}

int lbm_nn_cast_bf16(const float *x, size_t n, void *y, void *stream) {
    if (!x || !y) return LBM_NN_E_INVAL;
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid_for(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x, n, static_cast<bf16 *>(y));
    return check(hipGetLastError());
}

}  // extern "C"
