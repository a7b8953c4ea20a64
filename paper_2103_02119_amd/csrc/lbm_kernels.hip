// HIP kernels (gfx950) of the rectangular-lattice central-moment LBM
// (Yahia & Premnath, arXiv 2103.02119).
//
// Step kernel layout
//   * Populations live in 9 SoA planes [k][ny][pitch] (pitch = nx rounded up
//     to 64 values), x fastest, so a wavefront's 64 lanes read and write one
//     contiguous 64-value row segment per plane.
//   * Pull streaming: the step at time t reads the post-collision values of
//     t-1 shifted by (cx, cy) nodes (perfect shift, Sec. 3 / Sec. 4), so all
//     stores are aligned and coalesced.  A buffer that holds pre-collision
//     values (after set_fields / set_populations) is read in place instead.
//   * Each wavefront owns 64 columns x `rows` rows and marches up the rows,
//     keeping the populations of rows j and j+1 in registers.  The density
//     gradient (the only non-local input of the collision, Sec. 2.3) needs
//     rho of the 4 neighbours at the same time level: the row below and above
//     come from the marching window, the left/right neighbours from a
//     wavefront shuffle, and the two columns beyond the segment from a halo
//     pass done once per wavefront (one halo node per lane).
//   * The collision is done in component form (the paper's advice, Sec. 3):
//     1-D moment transforms along x then y, the relaxation in the paper's
//     moment basis, then the inverse transforms.  No matrix is formed.
//   * FP32 deviation mode stores g = f - w rho0 and carries every moment as a
//     deviation from the rest state so that no O(1) quantity is subtracted
//     from another in FP32.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------ small helpers

__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}

template <typename R>
__device__ __forceinline__ R sum9(const R (&f)[9]) {
    // same grouping as the x-sums of the collision: (0,1,3), (2,5,6), (4,8,7)
    return ((f[0] + f[1] + f[3]) + (f[2] + f[5] + f[6])) + (f[4] + f[8] + f[7]);
}

struct RowInfo {
    int j, jb, jt;   // row, source row of cy = +1 links, source row of cy = -1 links
    bool wb, wt;     // source of cy = +1 / cy = -1 links lies across a wall
};
struct ColInfo {
    int x, xl, xr;   // column, source column of cx = +1 links, of cx = -1 links
    bool wl, wr;
};

__device__ __forceinline__ RowInfo row_info(int j, const Geometry &G) {
    RowInfo r;
    const bool cb = (j == 0), ct = (j == G.ny - 1);
    r.j = j;
    r.jb = cb ? G.ny - 1 : j - 1;
    r.jt = ct ? 0 : j + 1;
    r.wb = cb && G.bc[kYmin] != kPeriodic;
    r.wt = ct && G.bc[kYmax] != kPeriodic;
    return r;
}
__device__ __forceinline__ ColInfo col_info(int x, const Geometry &G) {
    ColInfo c;
    const bool cl = (x == 0), cr = (x == G.nx - 1);
    c.x = x;
    c.xl = cl ? G.nx - 1 : x - 1;
    c.xr = cr ? 0 : x + 1;
    c.wl = cl && G.bc[kXmin] != kPeriodic;
    c.wr = cr && G.bc[kXmax] != kPeriodic;
    return c;
}

// Pre-collision populations of node (x, j): pulled with periodic wrap and
// half-way bounce-back, f_k = f~_opp(k)(x) - (feq_opp(k) - feq_k)(rho0, u_w),
// where the source node lies beyond a wall (Sec. 5.2), or f_k = f~_opp(k)(x)
// where it is a solid node of the obstacle mask (a wall at rest).  Without
// PULL the buffer already holds pre-collision values and is read in place.
// A solid node itself reads as the rest state.
template <typename S, typename R, bool PULL>
__device__ __forceinline__ void load_node(const S *__restrict__ src, const Geometry &G,
                                          const Consts<R> &K, const RowInfo &r,
                                          const ColInfo &c, R (&f)[9]) {
    const long long P = G.plane;
    const long long own = static_cast<long long>(r.j) * G.pitch + c.x;
    if (G.mask && G.mask[own]) {  // a solid node holds the rest state
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = K.rest[k];
        return;
    }
    if (!PULL) {
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = static_cast<R>(src[k * P + own]);
        return;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = cx_of(k), cy = cy_of(k);
        const int row = cy > 0 ? r.jb : (cy < 0 ? r.jt : r.j);
        const int col = cx > 0 ? c.xl : (cx < 0 ? c.xr : c.x);
        const bool wy = cy > 0 ? r.wb : (cy < 0 ? r.wt : false);
        const bool wx = cx > 0 ? c.wl : (cx < 0 ? c.wr : false);
        if (wx || wy) {
            const int xf = cx > 0 ? kXmin : kXmax;
            const int yf = cy > 0 ? kYmin : kYmax;
            const bool use_x =
                wx && (!wy || (G.bc[xf] == kMovingWall && G.bc[yf] != kMovingWall));
            const R d = use_x ? K.dwall[xf][k] : K.dwall[yf][k];
            f[k] = static_cast<R>(src[opp_of(k) * P + own]) - d;
        } else {
            const long long so = static_cast<long long>(row) * G.pitch + col;
            if (G.mask && G.mask[so])  // solid source: half-way bounce-back at rest
                f[k] = static_cast<R>(src[opp_of(k) * P + own]);
            else
                f[k] = static_cast<R>(src[k * P + so]);
        }
    }
}

// Buffer resources: a 128-bit descriptor held in scalar registers (base,
// byte range, data format 32) plus a 32-bit per-lane byte offset.  Accesses
// past the range read 0 / are dropped by the hardware instead of faulting.
constexpr int kBufFlags = 0x00020000;
// cache-policy bits of a non-temporal store (used when the two population
// buffers do not fit the Infinity Cache, so the stores need not stay there)
constexpr int kStoreNT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0),
                                             static_cast<int>(bytes), kBufFlags);
}
__device__ __forceinline__ float buf_load(float *, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                          uint32_t soff) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), static_cast<int>(soff), 0));
}
__device__ __forceinline__ double buf_load(double *, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                           uint32_t soff) {
    return __builtin_bit_cast(
        double, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(off), static_cast<int>(soff), 0));
}
template <int AUX>
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                          uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, static_cast<int>(off),
                                          static_cast<int>(soff), AUX);
}
template <int AUX>
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t off,
                                          uint32_t soff) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, static_cast<int>(off),
                                          static_cast<int>(soff), AUX);
}

// Interior node (1 <= x <= nx-2, 1 <= j <= ny-2): no wrap, no wall.  One
// descriptor covers the nine planes; the plane and row shift of each
// direction is a wavefront-uniform scalar offset, the column shift an
// immediate, so the only per-lane address is one 32-bit byte offset per row.
// Needs the whole buffer below 4 GiB (Geometry::buf_ok).
// XW = 1 / 2: the tile's first / last column lies on a wall face (x = 0 /
// x = nx - 1, not periodic), rows interior.  The lane on the wall (wlane)
// takes the half-way bounce-back of Eq. 57-59 for the three links that
// would come from outside, from three extra loads of its own node's
// opposite planes; every other lane is interior.
template <typename S, typename R, bool PULL, int XW = 0>
__device__ __forceinline__ void load_interior(const S *__restrict__ src, const Geometry &G,
                                              int j, int x, R (&f)[9],
                                              const Consts<R> *K = nullptr, bool wlane = false) {
    constexpr uint32_t B = sizeof(S);
    const uint32_t pb = static_cast<uint32_t>(G.plane) * B;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, 9u * pb);
    // byte offset of (x - 1, j): column shifts become immediates 0, B, 2B
    const uint32_t obm = static_cast<uint32_t>(j * G.pitch + x - 1) * B;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = PULL ? cx_of(k) : 0, cy = PULL ? cy_of(k) : 0;
        const uint32_t soff = static_cast<uint32_t>(k) * pb -
                              static_cast<uint32_t>(cy * G.pitch) * B;
        f[k] = static_cast<R>(buf_load(static_cast<S *>(nullptr), rs, obm + (1 - cx) * B, soff));
        if constexpr (PULL && XW != 0) {
            if (cx == (XW == 1 ? 1 : -1)) {
                const int face = XW == 1 ? kXmin : kXmax;
                const R bb = static_cast<R>(buf_load(static_cast<S *>(nullptr), rs, obm + B,
                                                     static_cast<uint32_t>(opp_of(k)) * pb));
                f[k] = wlane ? bb - K->dwall[face][k] : f[k];
            }
        }
    }
}

// load_interior for a node whose row and the rows it pulls from are interior
// but which may sit on the first or last column: a link from beyond an x
// face wraps (periodic: a per-lane shift of the column by nx) or bounces back
// half-way (wall: the node's own opposite population less the wall term of
// Eq. 57-59, from an extra load of its own opposite plane).
template <typename S, typename R, bool PULL>
__device__ __forceinline__ void load_edge(const S *__restrict__ src, const Geometry &G,
                                          const Consts<R> &K, int j, int x, R (&f)[9]) {
    constexpr uint32_t B = sizeof(S);
    const uint32_t pb = static_cast<uint32_t>(G.plane) * B;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, 9u * pb);
    const uint32_t obm = static_cast<uint32_t>(j * G.pitch + x - 1) * B;
    const bool left = x == 0, right = x == G.nx - 1;
    const bool lwall = left && G.bc[kXmin] != kPeriodic, rwall = right && G.bc[kXmax] != kPeriodic;
    const uint32_t wrap = static_cast<uint32_t>(G.nx) * B;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = PULL ? cx_of(k) : 0, cy = PULL ? cy_of(k) : 0;
        const uint32_t soff = static_cast<uint32_t>(k) * pb -
                              static_cast<uint32_t>(cy * G.pitch) * B;
        uint32_t voff = obm + (1 - cx) * B;
        if (cx == 1 && left && !lwall) voff += wrap;
        if (cx == -1 && right && !rwall) voff -= wrap;
        f[k] = static_cast<R>(buf_load(static_cast<S *>(nullptr), rs, voff, soff));
        if (cx != 0) {
            const bool w = cx == 1 ? lwall : rwall;
            const R bb = static_cast<R>(buf_load(static_cast<S *>(nullptr), rs, obm + B,
                                                 static_cast<uint32_t>(opp_of(k)) * pb));
            f[k] = w ? bb - K.dwall[cx == 1 ? kXmin : kXmax][k] : f[k];
        }
    }
}

template <typename S, typename R>
__device__ __forceinline__ void store_node(S *__restrict__ dst, const Geometry &G, int j, int x,
                                           const R (&o)[9]) {
    if (G.buf_ok) {
        constexpr uint32_t B = sizeof(S);
        const uint32_t pb = static_cast<uint32_t>(G.plane) * B;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(dst, 9u * pb);
        const uint32_t ob = static_cast<uint32_t>(j * G.pitch + x) * B;
        if (G.nt_store) {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                buf_store<kStoreNT>(static_cast<S>(o[k]), rs, ob, static_cast<uint32_t>(k) * pb);
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                buf_store<0>(static_cast<S>(o[k]), rs, ob, static_cast<uint32_t>(k) * pb);
        }
    } else {
        S *q = dst + static_cast<long long>(j) * G.pitch + x;
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k * G.plane] = static_cast<S>(o[k]);
    }
}

// ------------------------------------------------------------ collision

// 1-D inverse transform: central moments (k0, k1, k2) about velocity v of a
// 3-velocity set {0, +1, -1} -> populations (p0, p+, p-).
template <typename R>
__device__ __forceinline__ void inv1d(R k0, R k1, R k2, R v, R v2, R &p0, R &pp, R &pm) {
    const R r1 = k1 + v * k0;
    const R r2 = k2 + R(2) * v * k1 + v2 * k0;
    p0 = k0 - r2;
    pp = R(0.5) * (r2 + r1);
    pm = R(0.5) * (r2 - r1);
}

// Post-collision values o[9] of one node from its pre-collision values p[9]
// (f, or g = f - w rho0 in deviation mode) and the density gradient.
//   COLL == kRC : Sec. 4 (central moments, equilibria Eq. 49, sources
//                 (0, Fx, Fy, 0, ...), F / F^{-1} of App. B);
//   COLL == kRNR: Sec. 3 (raw moments, Eq. 12 with the m_8 coefficient 1,
//                 sources Eq. 13).
// Both add the corrections of Eq. 23-27 with the strain rate of Eq. 37-38.
// HU: omega_6 = omega_7 = omega_8 = 1 (the paper's setting), so the third-
// and fourth-order pre-collision moments are not needed.
// The work is split in two phases so that a step kernel can run the first
// (which does not need the density gradient) while the loads of the
// neighbouring row are still in flight.
// rho x with rho = rr + r00 kept split in deviation mode, so that the
// rounding of the density sum (see collide_pre) does not scale equilibrium
// terms by a regionally constant factor
template <bool DEV, typename R>
__device__ __forceinline__ R rho_times(R rr, R r00, R x) {
    return DEV ? rr * x + r00 * x : r00 * x;
}

template <typename R>
struct Pre {
    R r00, rho, irho, ux, uy, vy, vy2, ux2, uy2, uxuy;
    R N3, N4, N5, Q3, Q4, k20, k10;
};

template <typename R, bool DEV, int COLL>
__device__ __forceinline__ Pre<R> collide_pre(const R (&p)[9], const Consts<R> &K) {
    Pre<R> q;
    // x-sums of the three cy rows; (cx = 0, +1, -1) is (0,1,3), (2,5,6), (4,8,7)
    const R s0z = p[0] + p[1] + p[3], s1z = p[1] - p[3], s2z = p[1] + p[3];
    const R s0p = p[2] + p[5] + p[6], s1p = p[5] - p[6], s2p = p[5] + p[6];
    const R s0m = p[4] + p[8] + p[7], s1m = p[8] - p[7], s2m = p[8] + p[7];
    // raw moments r_mn = sum p cx^m cy^n (cy in units of a)
    const R r02 = s0p + s0m;
    const R r00 = s0z + r02;
    const R r10 = s1z + s1p + s1m;
    const R r20 = s2z + s2p + s2m;
    const R r01 = s0p - s0m;
    const R r11 = s1p - s1m;
    // macroscopic fields, rho u = sum f e + F/2
    const R rr = DEV ? K.rr : R(0);
    const R jx = r10 + K.hFx, jy = K.a * r01 + K.hFy;
    q.r00 = r00;
    q.rho = rr + r00;
    if (DEV && sizeof(R) == 4) {
        // In FP32 the sum rr + r00 drops the low bits of the density
        // deviation, and that rounding is the same over whole regions where
        // the density varies slowly: u = j / rho would carry a regionally
        // constant relative error, i.e. a momentum source or sink at every
        // collision.  One Newton step against the unrounded density
        // rr + r00 removes it (the residual j - u0 (rr + r00) is formed with
        // the two parts of the density separately).
        q.irho = __builtin_amdgcn_rcpf(q.rho);
        const R ux0 = jx * q.irho, uy0 = jy * q.irho;
        const R ex = __builtin_fmaf(-ux0, rr, jx) - ux0 * r00;
        const R ey = __builtin_fmaf(-uy0, rr, jy) - uy0 * r00;
        q.ux = __builtin_fmaf(ex, q.irho, ux0);
        q.uy = __builtin_fmaf(ey, q.irho, uy0);
    } else {
        q.irho = R(1) / q.rho;
        q.ux = jx * q.irho;
        q.uy = jy * q.irho;
    }
    q.ux2 = q.ux * q.ux;
    q.uy2 = q.uy * q.uy;
    q.uxuy = q.ux * q.uy;
    const R ux = q.ux, uy = q.uy, ux2 = q.ux2, uy2 = q.uy2;
    // second-order non-equilibrium parts N3, N4, N5 (f level, paper basis)
    // and the raw ones Q3, Q4 of Eq. 34-35 used by the strain rate
    if (COLL == kRC) {
        q.vy = uy * K.inv_a;  // velocity in units of a
        q.vy2 = q.vy * q.vy;
        q.k20 = r20 - R(2) * ux * r10 + ux2 * r00;            // sum p (cx-ux)^2
        const R k02 = r02 - R(2) * q.vy * r01 + q.vy2 * r00;  // sum p (cy-vy)^2
        q.k10 = r10 - ux * r00;
        const R k11 = (r11 - ux * r01) - q.vy * q.k10;        // sum p (cx-ux)(cy-vy)
        const R ak02 = K.a2 * k02;
        q.N3 = (q.k20 + ak02) - R(2) * K.s * r00 + rr * (ux2 + uy2);
        q.N4 = (q.k20 - ak02) + rr * (ux2 - uy2);
        q.N5 = K.a * k11 + rr * q.uxuy;
        q.Q3 = q.N3 - (ux * K.Fx + uy * K.Fy);
        q.Q4 = q.N4 - (ux * K.Fx - uy * K.Fy);
    } else {
        q.vy = R(0);
        q.vy2 = R(0);
        q.k20 = R(0);
        q.k10 = R(0);
        const R ar02 = K.a2 * r02;
        q.N3 = (r20 + ar02) - R(2) * K.s * r00 - rho_times<DEV>(rr, r00, ux2 + uy2);
        q.N4 = (r20 - ar02) - rho_times<DEV>(rr, r00, ux2 - uy2);
        q.N5 = K.a * r11 - rho_times<DEV>(rr, r00, q.uxuy);
        q.Q3 = q.N3;
        q.Q4 = q.N4;
    }
    return q;
}

template <typename R, bool DEV, int COLL, bool HU>
__device__ __forceinline__ void collide_post(const R (&p)[9], const Pre<R> &q, R gx, R gy,
                                             int corr, const Consts<R> &K, R (&o)[9]) {
    const R rr = DEV ? K.rr : R(0);
    const R rho = q.rho, ux = q.ux, uy = q.uy, ux2 = q.ux2, uy2 = q.uy2, uxuy = q.uxuy;
    const R r00 = q.r00;
    // local strain rate (Eq. 37-38, coefficients Eq. 40 divided by rho) and
    // the corrections (Eq. 23-26; Eq. 27: none on m_5)
    R del3 = R(0), del4 = R(0);
    if (corr) {
        const R tx = K.e1 * ux * gx;  // B3 d_x rho = C3 d_x rho
        const R ty = K.e2 * uy * gy;  // B4 d_y rho = -C4 d_y rho
        const R M3 = q.Q3 - tx - ty;
        const R M4 = q.Q4 - tx + ty;
        const R b1 = K.b1c + R(1.5) * ux2, b2 = K.b2c + R(1.5) * uy2;
        const R c1 = K.c1c + R(1.5) * ux2, c2 = K.c2c - R(1.5) * uy2;
        const R idet = q.irho / (b1 * c2 - c1 * b2);
        const R X = (c2 * M3 - b2 * M4) * idet;  // d ux / dx
        const R Y = (b1 * M4 - c1 * M3) * idet;  // d uy / dy
        const R t1 = K.q1 * (rho * X + ux * gx);
        const R t2 = K.q2 * (rho * Y + uy * gy);
        const R G3 = R(3) * rho * (ux2 * X + uy2 * Y);
        const R G4 = R(3) * rho * (ux2 * X - uy2 * Y);
        del3 = K.k3 * (t1 + t2 - G3);
        del4 = K.k4 * (t1 - t2 - G4);
    }

    // post-collision moments in the paper basis, as deviations from rr * rest
    R D0, D1, D2, D3, D4, D5, D6, D7, D8;
    const R sux2 = K.s + ux2, suy2 = K.s + uy2;
    if (COLL == kRC) {
        D0 = r00;
        D1 = K.hFx + rr * ux;  // relaxed first central moment = F/2 for any omega
        D2 = K.hFy + rr * uy;
        D3 = R(2) * K.s * r00 - rr * (ux2 + uy2) + K.om[3] * q.N3 + K.w[3] * del3;
        D4 = -rr * (ux2 - uy2) + K.om[4] * q.N4 + K.w[4] * del4;
        D5 = -rr * uxuy + K.om[5] * q.N5;
        if (HU) {
            D6 = rr * sux2 * uy;
            D7 = rr * ux * suy2;
            D8 = K.s2 * r00 - rr * (K.s * (ux2 + uy2) + ux2 * uy2);
        } else {
            const R s1p = p[5] - p[6], s2p = p[5] + p[6];
            const R s1m = p[8] - p[7], s2m = p[8] + p[7];
            const R s0p = p[2] + p[5] + p[6], s0m = p[4] + p[8] + p[7];
            const R r01 = s0p - s0m, r02 = s0p + s0m, r11 = s1p - s1m;
            const R r21 = s2p - s2m, r12 = s1p + s1m, r22 = s2p + s2m;
            const R vy = q.vy, vy2 = q.vy2;
            const R x21 = r21 - R(2) * ux * r11 + ux2 * r01;  // sum p (cx-ux)^2 cy
            const R x11 = r11 - ux * r01;                     // sum p (cx-ux) cy
            const R x12 = r12 - ux * r02;                     // sum p (cx-ux) cy^2
            const R x22 = r22 - R(2) * ux * r12 + ux2 * r02;  // sum p (cx-ux)^2 cy^2
            const R k21 = x21 - vy * q.k20;
            const R k12 = x12 - R(2) * vy * x11 + vy2 * q.k10;
            const R k22 = x22 - R(2) * vy * x21 + vy2 * q.k20;
            const R M6 = K.a * k21 - rr * sux2 * uy;
            const R M7 = K.a2 * k12 - rr * ux * suy2;
            const R M8 = K.a2 * k22 + rr * sux2 * suy2;
            D6 = K.om[6] * M6 + rr * sux2 * uy;
            D7 = K.om[7] * M7 + rr * ux * suy2;
            D8 = K.om[8] * M8 + K.w[8] * rho * K.s2 - rr * sux2 * suy2;
        }
    } else {
        const R Fx = K.Fx, Fy = K.Fy;
        const R phi3 = R(2) * (Fx * ux + Fy * uy);
        const R phi4 = R(2) * (Fx * ux - Fy * uy);
        const R phi5 = Fx * uy + Fy * ux;
        const R phi6 = Fy * ux2 + R(2) * Fx * uxuy;
        const R phi7 = Fx * uy2 + R(2) * Fy * uxuy;
        const R phi8 = R(2) * (Fx * ux * uy2 + Fy * uy * ux2);
        const R s0p = p[2] + p[5] + p[6], s0m = p[4] + p[8] + p[7];
        const R s1z = p[1] - p[3], s1p = p[5] - p[6], s1m = p[8] - p[7];
        D0 = r00;
        D1 = (s1z + s1p + s1m) + Fx;  // momentum gains F for any omega_1, omega_2
        D2 = K.a * (s0p - s0m) + Fy;
        D3 = R(2) * K.s * r00 + rho_times<DEV>(rr, r00, ux2 + uy2) + K.om[3] * q.N3 +
             K.w[3] * del3 + K.sw[3] * phi3;
        D4 = rho_times<DEV>(rr, r00, ux2 - uy2) + K.om[4] * q.N4 + K.w[4] * del4 + K.sw[4] * phi4;
        D5 = rho_times<DEV>(rr, r00, uxuy) + K.om[5] * q.N5 + K.sw[5] * phi5;
        const R e6 = rho_times<DEV>(rr, r00, uy * sux2), e7 = rho_times<DEV>(rr, r00, ux * suy2);
        const R e8x = r00 * K.s2 + rho_times<DEV>(rr, r00, K.s * (ux2 + uy2) + ux2 * uy2);  // eq8 - rr s^2
        if (HU) {
            D6 = e6 + R(0.5) * phi6;
            D7 = e7 + R(0.5) * phi7;
            D8 = e8x + R(0.5) * phi8;
        } else {
            const R s2p = p[5] + p[6], s2m = p[8] + p[7];
            const R r21 = s2p - s2m, r12 = s1p + s1m, r22 = s2p + s2m;
            const R N6 = K.a * r21 - e6;
            const R N7 = K.a2 * r12 - e7;
            const R N8 = K.a2 * r22 - e8x;
            D6 = e6 + K.om[6] * N6 + K.sw[6] * phi6;
            D7 = e7 + K.om[7] * N7 + K.sw[7] * phi7;
            D8 = e8x + K.om[8] * N8 + K.sw[8] * phi8;
        }
    }

    // back to natural moments in (cx, cy) units
    const R t20 = R(0.5) * (D3 + D4);
    const R t02 = R(0.5) * (D3 - D4) * K.inv_a2;
    const R t01 = D2 * K.inv_a, t11 = D5 * K.inv_a, t21 = D6 * K.inv_a;
    const R t12 = D7 * K.inv_a2, t22 = D8 * K.inv_a2;
    // RC: they are central moments about (ux, vy); RNR: raw (about 0)
    const R sx = (COLL == kRC) ? ux : R(0), sx2 = (COLL == kRC) ? ux2 : R(0);
    const R sy = (COLL == kRC) ? q.vy : R(0), sy2 = (COLL == kRC) ? q.vy2 : R(0);
    // y stage for m = 0, 1, 2
    R y00, y0p, y0m, y10, y1p, y1m, y20, y2p, y2m;
    inv1d(D0, t01, t02, sy, sy2, y00, y0p, y0m);
    inv1d(D1, t11, t12, sy, sy2, y10, y1p, y1m);
    inv1d(t20, t21, t22, sy, sy2, y20, y2p, y2m);
    // x stage for cy = 0, +1, -1
    inv1d(y00, y10, y20, sx, sx2, o[0], o[1], o[3]);
    inv1d(y0p, y1p, y2p, sx, sx2, o[2], o[5], o[6]);
    inv1d(y0m, y1m, y2m, sx, sx2, o[4], o[8], o[7]);
}

template <typename R, bool DEV, int COLL, bool HU>
__device__ __forceinline__ void collide(const R (&p)[9], R gx, R gy, int corr,
                                        const Consts<R> &K, R (&o)[9]) {
    const Pre<R> q = collide_pre<R, DEV, COLL>(p, K);
    collide_post<R, DEV, COLL, HU>(p, q, gx, gy, corr, K, o);
}

// ------------------------------------------------------------ step kernel

// Marches one wavefront tile (64 columns x rows j0..j1-1), keeping the
// populations of rows j .. j+D in registers: row j is collided while row
// j+D is in flight (D = 2; a deeper window measured slower for FP32 storage,
// where the last rows of a tile re-read the ring row more often, and the
// registers are scarce for FP64).  GENERIC handles wrap-around and walls on every
// load; the fast variant is used when every node the tile pulls is interior,
// so it carries no boundary logic and no wall constants.  The halo columns'
// populations arrive with the prologue and are summed only afterwards, so
// the tile starts with a single latency round.
// SMALL (fast path, tiles of exactly two rows): the prologue also loads the
// ring row above, so the whole tile arrives in one round of loads and the
// row steps issue none.
template <typename S, typename R, bool DEV, int COLL, bool PULL, bool HU, bool GENERIC, int XW = 0,
          bool SMALL = false>
__device__ __forceinline__ void march(const S *__restrict__ src, S *__restrict__ dst,
                                      const Geometry &G, const Consts<R> &K, int lane, int j0,
                                      int j1, int x0, int x, int xraw, int xlast, bool active,
                                      bool wall_left, bool wall_right) {
    constexpr int D = 2;
    const ColInfo c = col_info(x, G);
    // the lane whose outer neighbour is the wall (XW tiles); lanes past
    // nx - 1 repeat column nx - 1 and are not stored
    const bool wlane = XW == 1 ? (x == 0) : (XW == 2 ? (x == G.nx - 1) : false);
    auto load_row = [&](int jj, R (&f9)[9]) {
        if (GENERIC)
            load_node<S, R, PULL>(src, G, K, row_info(jj, G), c, f9);
        else
            load_interior<S, R, PULL, XW>(src, G, jj, x, f9, &K, wlane);
    };
    // a row index that exists (wrapping periodically) or -1 beyond a wall
    auto row_of = [&](int jj) -> int {
        if (jj < G.ny) return jj;
        return (GENERIC && G.bc[kYmax] != kPeriodic) ? -1 : jj - G.ny;
    };

    // halo loads: lane l fetches the nodes at (x0 - 1, j0 + l) and (xlast + 1, j0 + l)
    R hfl[9], hfr[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) hfl[k] = hfr[k] = R(0);
    {
        const int jh = min(j0 + lane, j1 - 1);
        const RowInfo rh = row_info(jh, G);
        // off the generic path the halo columns' own pulls stay inside the
        // lattice unless the right halo is the last column: buffer loads then
        if (!wall_left) {
            if (!GENERIC)
                load_interior<S, R, PULL>(src, G, jh, x0 - 1, hfl);
            else
                load_node<S, R, PULL>(src, G, K, rh, col_info(x0 > 0 ? x0 - 1 : G.nx - 1, G), hfl);
        }
        if (!wall_right) {
            if (!GENERIC && xlast + 2 < G.nx)
                load_interior<S, R, PULL>(src, G, jh, xlast + 1, hfr);
            else
                load_node<S, R, PULL>(src, G, K, rh, col_info(xlast < G.nx - 1 ? xlast + 1 : 0, G), hfr);
        }
    }
    // prologue: the ring row below and rows j0 .. j0 + D - 1
    const bool below = !GENERIC || (j0 > 0) || G.bc[kYmin] == kPeriodic;
    R fb[9];
    R fr[D + 1][9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        fb[k] = R(0);
#pragma unroll
        for (int d = 0; d <= D; ++d) fr[d][k] = R(0);
    }
    if (below) load_row(j0 > 0 ? j0 - 1 : G.ny - 1, fb);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (GENERIC) {
            const int jj = row_of(j0 + d);
            if (j0 + d <= j1 && jj >= 0) load_row(jj, fr[d]);
        } else {
            load_row(min(j0 + d, j1), fr[d]);
        }
    }
    if constexpr (SMALL) load_row(j0 + 2, fr[2]);
    const R hl = wall_left ? R(0) : sum9(hfl);
    const R hr = wall_right ? R(0) : sum9(hfr);
    R rc = sum9(fr[0]);
    R rb = below ? sum9(fb) : rc;  // wall: the missing neighbour's density is the node's own

    // One row: issue the loads of row j + D into `nxt` (the array that held
    // row j - 1), collide row j (`cur`) with the density of row j + 1 from
    // `up`.  The loop is unrolled D + 1 times with the arrays' roles permuted,
    // so no register that an in-flight load targets is ever copied (a copy
    // would make the wavefront wait for every outstanding load).
    auto row_step = [&](int j, R (&cur)[9], R (&up)[9], R (&nxt)[9]) {
        if constexpr (SMALL) {
        } else if (GENERIC) {
            const int jj = row_of(j + D);
            if (j + D <= j1 && jj >= 0) load_row(jj, nxt);
        } else {
            // unconditional (the last rows re-read the cached ring row j1): a
            // load inside a branch would make the wait counts collapse to a
            // full drain where the paths join
            load_row(min(j + D, j1), nxt);
        }
        const Pre<R> q = collide_pre<R, DEV, COLL>(cur, K);

        // densities of the four neighbours at the same time level
        const R rn = row_of(j + 1) >= 0 ? sum9(up) : rc;
        R rl = __shfl_up(rc, 1);
        R rgt = __shfl_down(rc, 1);
        const R hlj = readlane(hl, j - j0);
        const R hrj = readlane(hr, j - j0);
        if (lane == 0) rl = wall_left ? rc : hlj;
        if (xraw == xlast) rgt = wall_right ? rc : hrj;
        R rnu = rn, rbu = rb;
        bool solid = false;
        if (GENERIC && G.mask) {
            // a solid neighbour's density is replaced by the node's own (as at a wall)
            const unsigned char *m = G.mask;
            const long long ro = static_cast<long long>(j) * G.pitch;
            const int jn = row_of(j + 1);
            const int jb = j > 0 ? j - 1 : (G.bc[kYmin] == kPeriodic ? G.ny - 1 : -1);
            const int xl = x > 0 ? x - 1 : (G.bc[kXmin] == kPeriodic ? G.nx - 1 : -1);
            const int xr = x < G.nx - 1 ? x + 1 : (G.bc[kXmax] == kPeriodic ? 0 : -1);
            solid = m[ro + x] != 0;
            if (xl >= 0 && m[ro + xl]) rl = rc;
            if (xr >= 0 && m[ro + xr]) rgt = rc;
            if (jn >= 0 && m[static_cast<long long>(jn) * G.pitch + x]) rnu = rc;
            if (jb >= 0 && m[static_cast<long long>(jb) * G.pitch + x]) rbu = rc;
        }
        const R gx = (rgt - rl) * R(0.5);
        const R gy = (rnu - rbu) * K.half_inv_a;

        R out[9];
        collide_post<R, DEV, COLL, HU>(cur, q, gx, gy, G.corr, K, out);
        if (GENERIC && solid) {
#pragma unroll
            for (int k = 0; k < 9; ++k) out[k] = K.rest[k];
        }
        if (active) store_node(dst, G, j, xraw, out);
        rb = rc;
        rc = rn;
    };
    static_assert(D == 2, "the unrolled march below rotates three row arrays");
    for (int j = j0; j < j1; j += 3) {
        row_step(j, fr[0], fr[1], fr[2]);
        if (j + 1 < j1) row_step(j + 1, fr[1], fr[2], fr[0]);
        if (j + 2 < j1) row_step(j + 2, fr[2], fr[0], fr[1]);
    }
}

// One wavefront tile: 64 columns (segment seg) x G.rows rows (chunk).
// SMALL: the kernel instance for tiles of two rows (the paper's rates, pull
// form), whose fast paths load the whole tile in one round; kept in its own
// kernel so that its registers do not count against the general one.
template <typename S, typename R, bool DEV, int COLL, bool PULL, bool HU, bool SMALL = false>
__device__ __forceinline__ void run_tile(const S *__restrict__ src, S *__restrict__ dst,
                                         const Geometry &G, const Consts<R> &K, int lane, int seg,
                                         int chunk, bool near_solid) {
    const int x0 = seg * kWave;
    const int j0 = chunk * G.rows;
    const int j1 = min(j0 + G.rows, G.ny);
    const int xlast = min(x0 + kWave - 1, G.nx - 1);
    const int xraw = x0 + lane;
    const bool active = xraw < G.nx;
    const int x = min(xraw, G.nx - 1);
    const bool wall_left = (x0 == 0) && G.bc[kXmin] != kPeriodic;
    const bool wall_right = (xlast == G.nx - 1) && G.bc[kXmax] != kPeriodic;
    // every pulled node (rows j0-1 .. j1, columns x0-1 .. x0+64) interior
    // and fluid, or outside only across one x wall?  (the wall-column
    // variants only for the paper's omega_6..8 = 1, whose collision is small
    // enough for the extra registers)
    const bool rows_in = G.buf_ok && !near_solid && (j0 >= 2) && (j1 <= G.ny - 2) &&
                         (!SMALL || j1 - j0 == 2);
    const bool cols_in = (x0 > 0) && (x0 + kWave < G.nx);
    if (rows_in && cols_in)
        march<S, R, DEV, COLL, PULL, HU, false, 0, SMALL>(src, dst, G, K, lane, j0, j1, x0, x,
                                                          xraw, xlast, active, wall_left,
                                                          wall_right);
    else if (HU && rows_in && wall_left && x0 + kWave < G.nx)
        march<S, R, DEV, COLL, PULL, HU, false, HU ? 1 : 0, SMALL>(src, dst, G, K, lane, j0, j1,
                                                                   x0, x, xraw, xlast, active,
                                                                   wall_left, wall_right);
    else if (HU && rows_in && wall_right && x0 > 0)
        march<S, R, DEV, COLL, PULL, HU, false, HU ? 2 : 0, SMALL>(src, dst, G, K, lane, j0, j1,
                                                                   x0, x, xraw, xlast, active,
                                                                   wall_left, wall_right);
    else
        march<S, R, DEV, COLL, PULL, HU, true>(src, dst, G, K, lane, j0, j1, x0, x, xraw, xlast,
                                                active, wall_left, wall_right);
}

template <typename S, typename R, bool DEV, int COLL, bool PULL, bool HU, bool SMALL = false>
__global__ void __launch_bounds__(kBlock)
step_kernel(const S *__restrict__ src, S *__restrict__ dst, const Geometry G, const Consts<R> K) {
    const int lane = threadIdx.x & (kWave - 1);
    int b = blockIdx.x;
    // workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so neighbouring segments share its L2
    if (G.xcd_remap) b = (b & 7) * (G.nblocks >> 3) + (b >> 3);
    // the wavefront index is uniform across the wavefront; say so, so that all
    // tile bookkeeping lives in scalar registers and branches are scalar
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int tile = b * kWavesPerBlock + wave;
    if (tile >= G.ntile) return;
    const bool near_solid = G.tile_solid && G.tile_solid[tile];
    run_tile<S, R, DEV, COLL, PULL, HU, SMALL>(src, dst, G, K, lane, tile % G.nseg,
                                               tile / G.nseg, near_solid);
}

// Batched step: a persistent grid walks the tile list of all active cases
// (tiles of one case are contiguous).  The per-case geometry and constants
// are read from device tables with a wavefront-uniform case index, so they
// stay in scalar registers like kernel arguments.  The tile count lives in
// device memory, so a captured graph stays valid when the list changes.
template <typename S, typename R, bool DEV, int COLL, bool HU>
__global__ void __launch_bounds__(kBlock)
batch_step_kernel(S *__restrict__ buf0, S *__restrict__ buf1,
                  const BatchTile *__restrict__ tiles, const int *__restrict__ ntiles,
                  const BatchCase *__restrict__ cases, const Geometry *__restrict__ geoms,
                  const Consts<R> *__restrict__ Ks, int flip, int force_pull) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nb = static_cast<int>(gridDim.x);
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int n = *ntiles;
    for (int t = b * kWavesPerBlock + wave; t < n; t += nb * kWavesPerBlock) {
        const BatchTile td = tiles[t];
        const int c = __builtin_amdgcn_readfirstlane(td.c);
        const int seg = __builtin_amdgcn_readfirstlane(td.seg);
        const int chunk = __builtin_amdgcn_readfirstlane(td.chunk);
        const bool near_solid = __builtin_amdgcn_readfirstlane(td.pad) != 0;
        const Geometry &G = geoms[c];
        const Consts<R> &K = Ks[c];
        const int cur = __builtin_amdgcn_readfirstlane(cases[c].cur) ^ flip;
        // derived from the kernel's buffer arguments, so that the compiler
        // knows them to be global memory
        const long long off = cases[c].off;
        const S *src = (cur ? buf1 : buf0) + off;
        S *dst = (cur ? buf0 : buf1) + off;
        if (force_pull || cases[c].pull)
            run_tile<S, R, DEV, COLL, true, HU>(src, dst, G, K, lane, seg, chunk, near_solid);
        else
            run_tile<S, R, DEV, COLL, false, HU>(src, dst, G, K, lane, seg, chunk, near_solid);
    }
}

template <typename S, typename R, bool DEV>
static hipError_t batch_dispatch(int coll, bool hu, void *b0, void *b1, const BatchTile *tiles,
                                 const int *ntiles,
                                 const BatchCase *cases, const Geometry *geoms,
                                 const Consts<R> *K, int flip, int force_pull, int wgs,
                                 hipStream_t st) {
    const dim3 grid(wgs), block(kBlock);
#define LBM_BSTEP(C, H)                                                                  \
    hipLaunchKernelGGL((batch_step_kernel<S, R, DEV, C, H>), grid, block, 0, st,             \
                       static_cast<S *>(b0), static_cast<S *>(b1), tiles, ntiles, cases, geoms, \
                       K, flip, force_pull)
    if (coll == kRC) {
        if (hu) LBM_BSTEP(kRC, true); else LBM_BSTEP(kRC, false);
    } else {
        if (hu) LBM_BSTEP(kRNR, true); else LBM_BSTEP(kRNR, false);
    }
#undef LBM_BSTEP
    return hipGetLastError();
}

hipError_t launch_batch_step(int prec, int coll, bool hu, void *b0, void *b1,
                             const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                             const Geometry *geoms,
                             const Consts<double> *Kd, const Consts<float> *Kf, int flip,
                             int force_pull, int wgs, hipStream_t st) {
    switch (prec) {
    case kFP64: return batch_dispatch<double, double, false>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    case kFP32Dev: return batch_dispatch<float, float, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kf, flip, force_pull, wgs, st);
    case kFP64Dev: return batch_dispatch<double, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    case kFP32DevF64: return batch_dispatch<float, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ tile kernel

// Neighbour column / row of the density gradient: wrapped across a periodic
// face, -1 across a wall.
__device__ __forceinline__ int nb_col(int x, int d, const Geometry &G) {
    const int n = x + d;
    if (n < 0) return G.bc[kXmin] == kPeriodic ? G.nx - 1 : -1;
    if (n >= G.nx) return G.bc[kXmax] == kPeriodic ? 0 : -1;
    return n;
}
__device__ __forceinline__ int nb_row(int j, int d, const Geometry &G) {
    const int n = j + d;
    if (n < 0) return G.bc[kYmin] == kPeriodic ? G.ny - 1 : -1;
    if (n >= G.ny) return G.bc[kYmax] == kPeriodic ? 0 : -1;
    return n;
}

// One node per thread: a workgroup of TY wavefronts owns a tile of 64
// columns x TY rows.  Every thread pulls its node's populations and puts the
// node's density in an LDS tile; the densities of the one-node ring around
// the tile come from extra pulls by three of the wavefronts (the row below,
// the row above, the two columns).  After one barrier each thread forms the
// density gradient from LDS and collides.  Unlike the march there is no
// serial dependence between rows, so every load of the tile is in flight at
// once: the shape for lattices that fit the Infinity Cache.
template <typename S, typename R, bool DEV, int COLL, bool PULL, bool HU, int TY>
__device__ __forceinline__ void tile_body(const S *__restrict__ src, S *__restrict__ dst,
                                          const Geometry &G, const Consts<R> &K, int x0, int j0,
                                          R (&srho)[TY + 2][kWave + 2]) {
    const int tx = threadIdx.x & (kWave - 1);
    const int ty = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int nact = min(kWave, G.nx - x0), nrow = min(TY, G.ny - j0);
    const int tc = min(tx, nact - 1), tr = min(ty, nrow - 1);
    const int x = x0 + tc, j = j0 + tr;
    const bool active = tx < nact && ty < nrow;
    // every node pulled by the tile or its density ring in interior rows and
    // no mask: buffer loads, with the x faces handled per lane on the first
    // and last column tiles; anything else takes the generic loader
    const bool rows_in = G.buf_ok && !G.mask && j0 >= 2 && j0 + nrow + 1 < G.ny;
    const bool cols_in = x0 >= 2 && x0 + nact + 1 < G.nx;
    auto load = [&](int xx, int jj, R (&f)[9]) {
        if (rows_in && cols_in)
            load_interior<S, R, PULL>(src, G, jj, xx, f);
        else if (rows_in)
            load_edge<S, R, PULL>(src, G, K, jj, xx, f);
        else
            load_node<S, R, PULL>(src, G, K, row_info(jj, G), col_info(xx, G), f);
    };
    R f[9];
    load(x, j, f);
    // the density ring
    const int jb = nb_row(j0, -1, G), jt = nb_row(j0 + nrow - 1, 1, G);
    const int xl = nb_col(x0, -1, G), xr = nb_col(x0 + nact - 1, 1, G);
    R hb = R(0), ht = R(0), hc = R(0);
    if (ty == 0 && jb >= 0) {
        R h[9];
        load(x, jb, h);
        hb = sum9(h);
    }
    if (ty == nrow - 1 && jt >= 0) {
        R h[9];
        load(x, jt, h);
        ht = sum9(h);
    }
    // lanes 0 .. nrow-1: column xl, lanes 32 .. 32+nrow-1: column xr
    const int cw = nrow > 1 ? 1 : 0;
    const int hrow = j0 + (tx & 31);
    const bool hlane = ty == cw && (tx & 31) < nrow && ((tx < 32) ? xl >= 0 : xr >= 0);
    if (hlane) {
        R h[9];
        load(tx < 32 ? xl : xr, hrow, h);
        hc = sum9(h);
    }
    const R rc = sum9(f);
    srho[tr + 1][tc + 1] = rc;
    if (ty == 0 && jb >= 0) srho[0][tc + 1] = hb;
    if (ty == nrow - 1 && jt >= 0) srho[nrow + 1][tc + 1] = ht;
    if (hlane) srho[(tx & 31) + 1][tx < 32 ? 0 : nact + 1] = hc;
    __syncthreads();

    // neighbours' densities; across a wall, or on a solid node, the node's own
    const int nxl = nb_col(x, -1, G), nxr = nb_col(x, 1, G);
    const int nyb = nb_row(j, -1, G), nyt = nb_row(j, 1, G);
    R rl = nxl < 0 ? rc : srho[tr + 1][tc];
    R rgt = nxr < 0 ? rc : srho[tr + 1][tc + 2];
    R rbu = nyb < 0 ? rc : srho[tr][tc + 1];
    R rnu = nyt < 0 ? rc : srho[tr + 2][tc + 1];
    bool solid = false;
    if (G.mask) {
        const unsigned char *m = G.mask;
        solid = m[static_cast<long long>(j) * G.pitch + x] != 0;
        if (nxl >= 0 && m[static_cast<long long>(j) * G.pitch + nxl]) rl = rc;
        if (nxr >= 0 && m[static_cast<long long>(j) * G.pitch + nxr]) rgt = rc;
        if (nyb >= 0 && m[static_cast<long long>(nyb) * G.pitch + x]) rbu = rc;
        if (nyt >= 0 && m[static_cast<long long>(nyt) * G.pitch + x]) rnu = rc;
    }
    const R gx = (rgt - rl) * R(0.5);
    const R gy = (rnu - rbu) * K.half_inv_a;
    const Pre<R> q = collide_pre<R, DEV, COLL>(f, K);
    R out[9];
    collide_post<R, DEV, COLL, HU>(f, q, gx, gy, G.corr, K, out);
    if (solid) {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = K.rest[k];
    }
    if (active) store_node(dst, G, j, x, out);
}

template <typename S, typename R, bool DEV, int COLL, bool PULL, bool HU, int TY>
__global__ void __launch_bounds__(kWave * TY)
tile_step_kernel(const S *__restrict__ src, S *__restrict__ dst, const Geometry G,
                 const Consts<R> K, int ntx, int nty) {
    __shared__ R srho[TY + 2][kWave + 2];
    int b = blockIdx.x;
    const int nb = static_cast<int>(gridDim.x);
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    if (b >= ntx * nty) return;                             // padding workgroup (whole block)
    tile_body<S, R, DEV, COLL, PULL, HU, TY>(src, dst, G, K, (b % ntx) * kWave, (b / ntx) * TY,
                                             srho);
}

// Batched form: a persistent grid walks a list of 64 x TY block tiles of all
// active cases (BatchTile {case, tile column, tile row}); the LDS tile is
// reused, with a barrier between tiles.
template <typename S, typename R, bool DEV, int COLL, bool HU, int TY>
__global__ void __launch_bounds__(kWave * TY)
batch_tile_kernel(S *__restrict__ buf0, S *__restrict__ buf1, const BatchTile *__restrict__ tiles,
                  const int *__restrict__ ntiles, const BatchCase *__restrict__ cases,
                  const Geometry *__restrict__ geoms, const Consts<R> *__restrict__ Ks, int flip,
                  int force_pull) {
    __shared__ R srho[TY + 2][kWave + 2];
    const int n = *ntiles;
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const BatchTile td = tiles[t];
        const int c = __builtin_amdgcn_readfirstlane(td.c);
        const int tcol = __builtin_amdgcn_readfirstlane(td.seg);
        const int trow = __builtin_amdgcn_readfirstlane(td.chunk);
        const Geometry &G = geoms[c];
        const Consts<R> &K = Ks[c];
        const int cur = __builtin_amdgcn_readfirstlane(cases[c].cur) ^ flip;
        const long long off = cases[c].off;
        const S *src = (cur ? buf1 : buf0) + off;
        S *dst = (cur ? buf0 : buf1) + off;
        if (force_pull || cases[c].pull)
            tile_body<S, R, DEV, COLL, true, HU, TY>(src, dst, G, K, tcol * kWave, trow * TY, srho);
        else
            tile_body<S, R, DEV, COLL, false, HU, TY>(src, dst, G, K, tcol * kWave, trow * TY, srho);
        __syncthreads();  // the next tile reuses the LDS tile
    }
}

int tile_workgroups(const Geometry &G) {
    const int ty = G.tile_rows == 16 ? 16 : 8;
    const int n = ((G.nx + kWave - 1) / kWave) * ((G.ny + ty - 1) / ty);
    return (n + 7) / 8 * 8;
}

template <typename S, typename R, bool DEV>
static hipError_t batch_tile_dispatch(int coll, bool hu, void *b0, void *b1, const BatchTile *tiles,
                                      const int *ntiles, const BatchCase *cases,
                                      const Geometry *geoms, const Consts<R> *K, int flip,
                                      int force_pull, int wgs, hipStream_t st) {
    const dim3 grid(wgs), block(kWave * kBatchTileRows);
#define LBM_BTILE(C, H)                                                                          \
    hipLaunchKernelGGL((batch_tile_kernel<S, R, DEV, C, H, kBatchTileRows>), grid, block, 0, st,  \
                       static_cast<S *>(b0), static_cast<S *>(b1), tiles, ntiles, cases, geoms,   \
                       K, flip, force_pull)
    if (coll == kRC) {
        if (hu) LBM_BTILE(kRC, true); else LBM_BTILE(kRC, false);
    } else {
        if (hu) LBM_BTILE(kRNR, true); else LBM_BTILE(kRNR, false);
    }
#undef LBM_BTILE
    return hipGetLastError();
}

hipError_t launch_batch_tile(int prec, int coll, bool hu, void *b0, void *b1,
                             const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                             const Geometry *geoms, const Consts<double> *Kd,
                             const Consts<float> *Kf, int flip, int force_pull, int wgs,
                             hipStream_t st) {
    switch (prec) {
    case kFP64: return batch_tile_dispatch<double, double, false>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    case kFP32Dev: return batch_tile_dispatch<float, float, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kf, flip, force_pull, wgs, st);
    case kFP64Dev: return batch_tile_dispatch<double, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    case kFP32DevF64: return batch_tile_dispatch<float, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, force_pull, wgs, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename S, typename R, bool DEV>
static hipError_t step_dispatch(int coll, bool pull, bool hu, const void *src, void *dst,
                                const Geometry &G, const Consts<R> &K, hipStream_t st) {
    const dim3 grid(G.nblocks), block(kBlock);
    const S *s = static_cast<const S *>(src);
    S *d = static_cast<S *>(dst);
    if (uses_tile_kernel(G)) {
        const int ntx = (G.nx + kWave - 1) / kWave, ty = G.tile_rows == 16 ? 16 : 8;
        const int nty = (G.ny + ty - 1) / ty;
        const dim3 tgrid(tile_workgroups(G)), tblock(kWave * ty);
#define LBM_TSTEP(C, P, H)                                                                        \
    do {                                                                                          \
        if (ty == 16)                                                                             \
            hipLaunchKernelGGL((tile_step_kernel<S, R, DEV, C, P, H, 16>), tgrid, tblock, 0, st, s, \
                               d, G, K, ntx, nty);                                                \
        else                                                                                      \
            hipLaunchKernelGGL((tile_step_kernel<S, R, DEV, C, P, H, 8>), tgrid, tblock, 0, st, s,  \
                               d, G, K, ntx, nty);                                                \
    } while (0)
        if (coll == kRC) {
            if (pull) { if (hu) LBM_TSTEP(kRC, true, true); else LBM_TSTEP(kRC, true, false); }
            else { if (hu) LBM_TSTEP(kRC, false, true); else LBM_TSTEP(kRC, false, false); }
        } else {
            if (pull) { if (hu) LBM_TSTEP(kRNR, true, true); else LBM_TSTEP(kRNR, true, false); }
            else { if (hu) LBM_TSTEP(kRNR, false, true); else LBM_TSTEP(kRNR, false, false); }
        }
#undef LBM_TSTEP
        return hipGetLastError();
    }
#define LBM_STEP(C, P, H) \
    hipLaunchKernelGGL((step_kernel<S, R, DEV, C, P, H>), grid, block, 0, st, s, d, G, K)
    // the two-row kernel pays off with FP32 arithmetic only (measured: 13.5 vs
    // 13.7 us on the 512 x 1024 cavity; 10% slower in FP64)
    if constexpr (sizeof(R) == 4) {
        if (pull && hu && G.rows == 2) {
            if (coll == kRC)
                hipLaunchKernelGGL((step_kernel<S, R, DEV, kRC, true, true, true>), grid, block, 0, st, s, d, G, K);
            else
                hipLaunchKernelGGL((step_kernel<S, R, DEV, kRNR, true, true, true>), grid, block, 0, st, s, d, G, K);
            return hipGetLastError();
        }
    }
    if (coll == kRC) {
        if (pull) {
            if (hu) LBM_STEP(kRC, true, true); else LBM_STEP(kRC, true, false);
        } else {
            if (hu) LBM_STEP(kRC, false, true); else LBM_STEP(kRC, false, false);
        }
    } else {
        if (pull) {
            if (hu) LBM_STEP(kRNR, true, true); else LBM_STEP(kRNR, true, false);
        } else {
            if (hu) LBM_STEP(kRNR, false, true); else LBM_STEP(kRNR, false, false);
        }
    }
#undef LBM_STEP
    return hipGetLastError();
}

hipError_t launch_step(int prec, int coll, bool pull, bool hu, const void *src, void *dst,
                       const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                       hipStream_t st) {
    switch (prec) {
    case kFP64: return step_dispatch<double, double, false>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32Dev: return step_dispatch<float, float, true>(coll, pull, hu, src, dst, G, Kf, st);
    case kFP64Dev: return step_dispatch<double, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32DevF64: return step_dispatch<float, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    default: return hipErrorInvalidValue;
    }
}

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
// separate kernels give.
template <typename S, bool PC, bool PP>
__global__ void __launch_bounds__(kReduceBlock)
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
