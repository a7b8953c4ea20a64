// Device code shared by the step kernels of the rectangular-lattice
// central-moment LBM (Yahia & Premnath, arXiv 2103.02119): node loaders with
// periodic wrap and half-way bounce-back, buffer-addressed loads and stores,
// and the collision in component form.
//
// Layout and conventions
//   * Populations live in 9 SoA planes [k][ny][pitch] (pitch = nx rounded up
//     to 64 values), x fastest, so a wavefront's 64 lanes read and write one
//     contiguous 64-value row segment per plane.
//   * Pull streaming: the step at time t reads the post-collision values of
//     t-1 shifted by (cx, cy) nodes (perfect shift, Sec. 3 / Sec. 4), so all
//     stores are aligned and coalesced.  A buffer that holds pre-collision
//     values (after set_fields / set_populations) is read in place instead.
//   * The collision is done in component form (the paper's advice, Sec. 3):
//     1-D moment transforms along x then y, the relaxation in the paper's
//     moment basis, then the inverse transforms.  No matrix is formed.
//   * FP32 deviation mode stores g = f - w rho0 and carries every moment as a
//     deviation from the rest state so that no O(1) quantity is subtracted
//     from another in FP32.
#pragma once

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

// Choice between two wavefront-uniform constants by a per-lane condition,
// made on the values: both are pinned in scalar registers first, so the
// compiler cannot turn the choice into a choice of address inside the
// kernel's constant arguments (which would make it copy them to private
// memory).
template <typename R>
__device__ __forceinline__ R pick_value(bool c, R a, R b) {
    asm volatile("" : "+s"(a));
    asm volatile("" : "+s"(b));
    return c ? a : b;
}

// Pre-collision populations of node (x, j): pulled with periodic wrap and
// half-way bounce-back, f_k = f~_opp(k)(x) - (feq_opp(k) - feq_k)(rho0, u_w),
// where the source node lies beyond a wall (Sec. 5.2), or f_k = f~_opp(k)(x)
// where it is a solid node of the obstacle mask (a wall at rest).  Without
// PULL the buffer already holds pre-collision values and is read in place.
// A solid node itself reads as the rest state.
// PIN: take the wall term through pick_value (for kernels that inline this
// loader in several code paths, where the compiler would otherwise choose
// between addresses of the constants); the one-path kernels keep the plain
// choice, which costs no extra register.
template <typename S, typename R, bool PULL, bool PIN = false>
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
            const R d = PIN ? pick_value(use_x, K.dwall[xf][k], K.dwall[yf][k])
                            : (use_x ? K.dwall[xf][k] : K.dwall[yf][k]);
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
// 3-velocity set {0, +1, -1} -> populations (p0, p+, p-), with the raw
// moments r1 = k1 + v k0, r2 = k2 + 2 v k1 + v^2 k0 and
// p0 = k0 - r2, p+- = (r2 +- r1) / 2.  The first and second moments come
// in halved (h1 = k1 / 2, h2 = k2 / 2) and so do v and v^2 where they scale
// k0 (hv = v / 2, hv2 = v^2 / 2; tv = 2 v): the halves of r1 and r2 then give
// p+- with one addition each.  Halving is exact in binary floating point,
// so every result equals that of the unhalved form bit for bit.
template <typename R>
__device__ __forceinline__ void inv1d(R k0, R h1, R h2, R hv, R hv2, R tv, R &p0, R &pp,
                                      R &pm) {
    const R g1 = h1 + hv * k0;               // r1 / 2
    const R g2 = (h2 + tv * h1) + hv2 * k0;  // r2 / 2
    p0 = k0 - R(2) * g2;
    pp = g2 + g1;
    pm = g2 - g1;
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
        // FP32: the hardware reciprocal (1 ulp) in place of an IEEE division,
        // which costs about ten instructions per node
        R idet;
        if constexpr (sizeof(R) == 4)
            idet = q.irho * __builtin_amdgcn_rcpf(b1 * c2 - c1 * b2);
        else
            idet = q.irho / (b1 * c2 - c1 * b2);
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

    // back to natural moments t_mn in (cx, cy) units: t00 = D0, t10 = D1,
    // t20 = (D3 + D4) / 2, t01 = D2 / a, t11 = D5 / a, t21 = D6 / a,
    // t02 = (D3 - D4) / (2 a^2), t12 = D7 / a^2, t22 = D8 / a^2.
    // The y stage takes t_m1, t_m2 halved; its outputs for m = 1, 2 are the
    // x stage's first and second moments, so those two rows go in scaled by
    // a further 1/2 (see inv1d).
    const R h_a = R(0.5) * K.inv_a;
    const R q_a = R(0.25) * K.inv_a, q_a2 = R(0.25) * K.inv_a2;
    const R h01 = D2 * h_a, h02 = (D3 - D4) * q_a2;                        // m = 0
    const R h10 = R(0.5) * D1, h11 = D5 * q_a, h12 = D7 * q_a2;             // m = 1, / 2
    const R h20 = R(0.25) * (D3 + D4), h21 = D6 * q_a, h22 = D8 * q_a2;     // m = 2, / 2
    // RC: they are central moments about (ux, vy); RNR: raw (about 0)
    const R sx = (COLL == kRC) ? ux : R(0), sx2 = (COLL == kRC) ? ux2 : R(0);
    const R sy = (COLL == kRC) ? q.vy : R(0), sy2 = (COLL == kRC) ? q.vy2 : R(0);
    const R hsx = R(0.5) * sx, hsx2 = R(0.5) * sx2, tsx = R(2) * sx;
    const R hsy = R(0.5) * sy, hsy2 = R(0.5) * sy2, tsy = R(2) * sy;
    // y stage for m = 0, 1, 2
    R y00, y0p, y0m, y10, y1p, y1m, y20, y2p, y2m;
    inv1d(D0, h01, h02, hsy, hsy2, tsy, y00, y0p, y0m);
    inv1d(h10, h11, h12, hsy, hsy2, tsy, y10, y1p, y1m);
    inv1d(h20, h21, h22, hsy, hsy2, tsy, y20, y2p, y2m);
    // x stage for cy = 0, +1, -1 (y1., y2. are halved moments)
    inv1d(y00, y10, y20, hsx, hsx2, tsx, o[0], o[1], o[3]);
    inv1d(y0p, y1p, y2p, hsx, hsx2, tsx, o[2], o[5], o[6]);
    inv1d(y0m, y1m, y2m, hsx, hsx2, tsx, o[4], o[8], o[7]);
}

template <typename R, bool DEV, int COLL, bool HU>
__device__ __forceinline__ void collide(const R (&p)[9], R gx, R gy, int corr,
                                        const Consts<R> &K, R (&o)[9]) {
    const Pre<R> q = collide_pre<R, DEV, COLL>(p, K);
    collide_post<R, DEV, COLL, HU>(p, q, gx, gy, corr, K, o);
}

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

}  // namespace lbm
