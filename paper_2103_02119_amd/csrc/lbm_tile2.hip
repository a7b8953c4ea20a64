// Two collide-and-stream steps per launch (temporal blocking) for lattices
// without an obstacle mask.
//
// One step reads 9 and writes 9 values per node, so a lattice larger than
// the Infinity Cache is bound by HBM at that traffic.  This kernel reads the
// populations of step t-1 once, keeps the post-collision values of step t of
// its tile in LDS and writes only those of step t+1: 9 reads and 9 writes per
// node for two lattice updates.
//
// Dependencies of one step (Sec. 3 / Sec. 4 algorithms): the post-collision
// values of a node need its pulled pre-collision values (the 8 neighbours'
// post-collision values of the previous step, perfect shift) and the
// densities of its 4 axis neighbours at the same time level (central
// differences, Sec. 2.3), which are themselves sums of pulled values.  So a
// node at step t+1 depends on the step-t state within two nodes, and on the
// step t-1 state within four.  For an output tile of 64 x TY nodes
// (x0 .. x0+63, j0 .. j0+TY-1) the workgroup
//   A  pulls the step-t pre-collision values of region Q = the tile grown by
//      3 nodes (70 x (TY+6)) from the source buffer and puts each density in
//      LDS;
//   B  collides the inner region P = the tile grown by 2 nodes (68 x (TY+4);
//      density gradient from LDS) and writes its post-collision values of
//      step t to an LDS tile;
//   C  pulls the step-t+1 pre-collision values of the tile and its one-node
//      density ring from that LDS tile (half-way bounce-back at walls) and
//      puts the densities in LDS;
//   D  collides the tile and stores step t+1 to the destination buffer.
// Neighbouring tiles recompute the overlap of their P regions: (68 (TY+4) +
// 64 TY) / (128 TY) collisions per lattice update, 1.30 at TY = 8 and 1.12
// at TY = 24.  Their reads of the overlapping halo rows and columns are
// served by L2 and the Infinity Cache.
//
// Two forms.  The register form (tile2_step_kernel, 64 TY threads) keeps
// the step-t pre-collision values of P in registers from A to B (at most two
// nodes per thread) and the step-t values in LDS in the storage type.  The
// staged form (tile2_staged_kernel) also parks the pre-collision values of P
// in the LDS tile, so no thread holds populations across a barrier and fewer
// threads than nodes can cover a taller tile, which recomputes less overlap.
//
// Periodic faces are handled by computing halo nodes with wrapped
// coordinates (the LDS tile is unwrapped, so steps B-D need no wrap), walls
// by leaving out the nodes beyond them and bouncing back the links that
// would come from there.  Every node goes through the same loaders,
// collision and rounding as in the one-step kernels (the step-t values are
// rounded to the storage type before step t+1 reads them), so two steps here
// equal two one-step launches bit for bit.
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

namespace {

template <int TY>
struct T2 {
    static constexpr int OW = kWave;       // output tile width
    static constexpr int PW = OW + 4;      // region P (step-t collisions)
    static constexpr int PH = TY + 4;
    static constexpr int QW = OW + 6;      // region Q (step-t densities)
    static constexpr int QH = TY + 6;
    static constexpr int CW = OW + 2;      // tile + its density ring (step t+1)
    static constexpr int CH = TY + 2;
    static constexpr int NT = kWave * TY;  // threads
    static constexpr int NP = PW * PH;     // P nodes
    static constexpr int NQR = 2 * QW + 2 * PH;  // Q nodes outside P
    static constexpr int NCR = 2 * CW + 2 * TY;  // ring nodes of the tile
    static_assert(NP <= 2 * NT, "at most two P nodes per thread");
    static_assert(NQR <= 2 * NT - NP, "the Q ring fits the threads with one P node");
    static_assert(NCR <= NT, "one ring node per thread");
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
    int m = v % n;
    return m < 0 ? m + n : m;
}

// A node of the (unwrapped) tile frame at global column x / row j: its
// wrapped coordinates and whether it exists (a node beyond a wall does not).
struct NodeAt {
    int x, j;
    bool in;
};
__device__ __forceinline__ NodeAt node_at(int x, int j, const Geometry &G) {
    NodeAt n;
    const bool px = G.bc[kXmin] == kPeriodic, py = G.bc[kYmin] == kPeriodic;
    n.in = (px || (x >= 0 && x < G.nx)) && (py || (j >= 0 && j < G.ny));
    n.x = px ? wrap_mod(x, G.nx) : x;
    n.j = py ? wrap_mod(j, G.ny) : j;
    return n;
}

// Pre-collision values of step t+1 of a node pulled from the step-t tile in
// LDS, pb[k][py][px] (the node at px, py of the P frame; global column x,
// row j).  WALLS: a link whose source lies beyond a wall bounces back
// half-way, f_k = f~_opp(k)(x) - (feq_opp(k) - feq_k)(rho0, u_w) (Sec. 5.2,
// Eq. 57-59), with the corner rule of the one-step loaders.
template <typename S, typename R, int PW, int PH, bool WALLS>
__device__ __forceinline__ void pull_lds(const S (*pb)[PH][PW], int px, int py, int x, int j,
                                         const Geometry &G, const Consts<R> &K, R (&f)[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = cx_of(k), cy = cy_of(k);
        const R v = static_cast<R>(pb[k][py - cy][px - cx]);
        if constexpr (WALLS) {
            const bool wx = (cx > 0 && x == 0 && G.bc[kXmin] != kPeriodic) ||
                            (cx < 0 && x == G.nx - 1 && G.bc[kXmax] != kPeriodic);
            const bool wy = (cy > 0 && j == 0 && G.bc[kYmin] != kPeriodic) ||
                            (cy < 0 && j == G.ny - 1 && G.bc[kYmax] != kPeriodic);
            if (wx || wy) {
                const int xf = cx > 0 ? kXmin : kXmax;
                const int yf = cy > 0 ? kYmin : kYmax;
                const bool use_x =
                    wx && (!wy || (G.bc[xf] == kMovingWall && G.bc[yf] != kMovingWall));
                const R d = pick_value(use_x, K.dwall[xf][k], K.dwall[yf][k]);
                f[k] = static_cast<R>(pb[opp_of(k)][py][px]) - d;
            } else {
                f[k] = v;
            }
        } else {
            f[k] = v;
        }
    }
}

// Densities of the four axis neighbours of a node for its gradient, from an
// LDS density tile rr[][W] at (lx, ly); across a wall the node's own (the
// zero-normal-gradient reading at a half-way wall).
template <typename R, int W, bool WALLS>
__device__ __forceinline__ void gradient(const R (*rr)[W], int lx, int ly, R rc, int x, int j,
                                         const Geometry &G, const Consts<R> &K, R &gx, R &gy) {
    R rl = rr[ly][lx - 1], rg = rr[ly][lx + 1], rb = rr[ly - 1][lx], rt = rr[ly + 1][lx];
    if constexpr (WALLS) {
        if (nb_col(x, -1, G) < 0) rl = rc;
        if (nb_col(x, 1, G) < 0) rg = rc;
        if (nb_row(j, -1, G) < 0) rb = rc;
        if (nb_row(j, 1, G) < 0) rt = rc;
    }
    gx = (rg - rl) * R(0.5);
    gy = (rt - rb) * K.half_inv_a;
}

// A node of the tile frame (interior tiles need no wrap and meet no wall).
template <int LOAD>
__device__ __forceinline__ NodeAt node_in(int x, int j, const Geometry &G) {
    if constexpr (LOAD == 0) return NodeAt{x, j, true};
    else return node_at(x, j, G);
}

// The step-t pre-collision values of node (x, j), pulled from the source
// buffer by the loader of the tile's class.
template <typename S, typename R, int LOAD>
__device__ __forceinline__ void load_any(const S *__restrict__ src, const Geometry &G,
                                         const Consts<R> &K, int x, int j, R (&f)[9]) {
    if constexpr (LOAD == 0)
        load_interior<S, R, true>(src, G, j, x, f);
    else if constexpr (LOAD == 1)
        load_edge<S, R, true>(src, G, K, j, x, f);
    else
        load_node<S, R, true, true>(src, G, K, row_info(j, G), col_info(x, G), f);
}

// LOAD: 0 = every pulled node interior (buffer loads, one offset per node),
// 1 = rows interior, columns wrap or meet an x wall (per-lane handling of the
// x faces), 2 = anything (generic loader).  WALLS: some face is a wall.
template <typename S, typename R, bool DEV, int COLL, bool HU, int TY, int LOAD, bool WALLS>
__device__ __forceinline__ void tile2_body(const S *__restrict__ src, S *__restrict__ dst,
                                           const Geometry &G, const Consts<R> &K, int x0, int j0,
                                           S (*pb)[T2<TY>::PH][T2<TY>::PW],
                                           R (*r1)[T2<TY>::QW], R (*r2)[T2<TY>::CW]) {
    using C = T2<TY>;
    const int t = static_cast<int>(threadIdx.x);

#define at(xx, jj) node_in<LOAD>(xx, jj, G)
#define load(xx, jj, f) load_any<S, R, LOAD>(src, G, K, xx, jj, f)

    // ---- A: step-t pre-collision values of P (registers) and densities of Q
    const int p0 = t, p1 = t + C::NT;
    const bool has1 = p1 < C::NP;
    // P frame (px, py) -> global (x0 - 2 + px, j0 - 2 + py)
    const int px0 = p0 % C::PW, py0 = p0 / C::PW;
    const int px1 = p1 % C::PW, py1 = p1 / C::PW;
    const NodeAt n0 = at(x0 - 2 + px0, j0 - 2 + py0);
    const NodeAt n1 = at(x0 - 2 + px1, j0 - 2 + py1);
    R f0[9], f1[9];
    if (LOAD == 0 || n0.in) load(n0.x, n0.j, f0);
    if (has1 && (LOAD == 0 || n1.in)) load(n1.x, n1.j, f1);
    // the Q nodes outside P: threads without a second P node, one each
    const int q = t - (C::NP - C::NT);
    const bool hasq = !has1 && q >= 0 && q < C::NQR;
    int qx = 0, qy = 0;
    if (q < C::QW) {
        qx = q;
        qy = 0;
    } else if (q < 2 * C::QW) {
        qx = q - C::QW;
        qy = C::QH - 1;
    } else if (q < 2 * C::QW + C::PH) {
        qx = 0;
        qy = 1 + q - 2 * C::QW;
    } else {
        qx = C::QW - 1;
        qy = 1 + q - 2 * C::QW - C::PH;
    }
    const NodeAt nq = at(x0 - 3 + qx, j0 - 3 + qy);
    if (hasq) {
        R h[9];
        if (LOAD == 0 || nq.in) {
            load(nq.x, nq.j, h);
            r1[qy][qx] = sum9(h);
        } else {
            r1[qy][qx] = R(0);
        }
    }
    // (a node beyond a wall has no values; its density slot holds 0 and is
    // never read by a gradient, which takes the node's own density there)
    const R rc0 = (LOAD == 0 || n0.in) ? sum9(f0) : R(0);
    const R rc1 = has1 && (LOAD == 0 || n1.in) ? sum9(f1) : R(0);
    r1[py0 + 1][px0 + 1] = rc0;
    if (has1) r1[py1 + 1][px1 + 1] = rc1;
    __syncthreads();

    // ---- B: collide P, step-t post-collision values to LDS
    {
        R gx, gy, o[9];
        if (LOAD == 0 || n0.in) {
            gradient<R, C::QW, WALLS>(r1, px0 + 1, py0 + 1, rc0, n0.x, n0.j, G, K, gx, gy);
            const Pre<R> pr = collide_pre<R, DEV, COLL>(f0, K);
            collide_post<R, DEV, COLL, HU>(f0, pr, gx, gy, G.corr, K, o);
#pragma unroll
            for (int k = 0; k < 9; ++k) pb[k][py0][px0] = static_cast<S>(o[k]);
        }
        if (has1 && (LOAD == 0 || n1.in)) {
            gradient<R, C::QW, WALLS>(r1, px1 + 1, py1 + 1, rc1, n1.x, n1.j, G, K, gx, gy);
            const Pre<R> pr = collide_pre<R, DEV, COLL>(f1, K);
            collide_post<R, DEV, COLL, HU>(f1, pr, gx, gy, G.corr, K, o);
#pragma unroll
            for (int k = 0; k < 9; ++k) pb[k][py1][px1] = static_cast<S>(o[k]);
        }
    }
    __syncthreads();

    // ---- C: step-t+1 pre-collision values of the tile (registers) and the
    // densities of the tile and its ring (LDS, in the space of r1)
    const int tx = t & (kWave - 1);
    const int ty = t >> 6;
    const int ox = x0 + tx, oj = j0 + ty;
    const NodeAt no = at(ox, oj);
    const bool active = ox < G.nx && oj < G.ny;
    R g[9];
    R rco = R(0);
    if (LOAD == 0 || no.in) {
        pull_lds<S, R, C::PW, C::PH, WALLS>(pb, tx + 2, ty + 2, no.x, no.j, G, K, g);
        rco = sum9(g);
    }
    // ring of the tile: rows j0 - 1 and j0 + TY (66 each), columns x0 - 1 and
    // x0 + 64 (TY each), in the C frame (origin x0 - 1, j0 - 1)
    int cx = 0, cy = 0;
    if (t < C::CW) {
        cx = t;
        cy = 0;
    } else if (t < 2 * C::CW) {
        cx = t - C::CW;
        cy = C::CH - 1;
    } else if (t < 2 * C::CW + TY) {
        cx = 0;
        cy = 1 + t - 2 * C::CW;
    } else {
        cx = C::CW - 1;
        cy = 1 + t - 2 * C::CW - TY;
    }
    const bool hasc = t < C::NCR;
    const NodeAt nc = at(x0 - 1 + cx, j0 - 1 + cy);
    R rcr = R(0);
    if (hasc && (LOAD == 0 || nc.in)) {
        R h[9];
        pull_lds<S, R, C::PW, C::PH, WALLS>(pb, cx + 1, cy + 1, nc.x, nc.j, G, K, h);
        rcr = sum9(h);
    }
    // r2 aliases r1: every read of r1 (step B) is behind the last barrier
    r2[ty + 1][tx + 1] = rco;
    if (hasc) r2[cy][cx] = rcr;
    __syncthreads();

    // ---- D: collide the tile, step t+1 to the destination buffer
    if (active && (LOAD == 0 || no.in)) {
        R gx, gy, o[9];
        gradient<R, C::CW, WALLS>(r2, tx + 1, ty + 1, rco, no.x, no.j, G, K, gx, gy);
        const Pre<R> pr = collide_pre<R, DEV, COLL>(g, K);
        collide_post<R, DEV, COLL, HU>(g, pr, gx, gy, G.corr, K, o);
        store_node(dst, G, oj, ox, o);
    }
#undef at
#undef load
}

// Staged form: the step-t pre-collision values of P wait in the LDS tile
// (each P node's slots are then overwritten by its own post-collision values
// in B), and NT threads cover a 64 x TY tile, TY * 64 / NT output rows per
// thread.  The tile holds the values in the arithmetic type; the
// post-collision ones are rounded to the storage type first, as if they had
// been stored and reloaded.
template <int TY, int NT>
struct T2S {
    static constexpr int OW = kWave;
    static constexpr int PW = OW + 4, PH = TY + 4;      // region P
    static constexpr int QW = OW + 6, QH = TY + 6;      // region Q
    static constexpr int CW = OW + 2, CH = TY + 2;      // tile + ring
    static constexpr int NQ = QW * QH, NP = PW * PH;
    static constexpr int QPER = (NQ + NT - 1) / NT;     // Q nodes per thread
    static constexpr int PPER = (NP + NT - 1) / NT;     // P nodes per thread
    static constexpr int WAVES = NT / kWave;
    static constexpr int RPT = TY / WAVES;              // output rows per thread
    static constexpr int NCR = 2 * CW + 2 * TY;         // ring nodes of the tile
    static_assert(NT % kWave == 0 && TY % WAVES == 0, "whole output rows per wavefront");
    static_assert(NCR <= NT, "one ring node per thread");
};

template <typename S, typename R, bool DEV, int COLL, bool HU, int TY, int NT, int LOAD, bool WALLS>
__device__ __forceinline__ void tile2_body_staged(const S *__restrict__ src, S *__restrict__ dst,
                                                  const Geometry &G, const Consts<R> &K, int x0,
                                                  int j0, R (*pb)[T2S<TY, NT>::PH][T2S<TY, NT>::PW],
                                                  R (*r1)[T2S<TY, NT>::QW],
                                                  R (*r2)[T2S<TY, NT>::CW]) {
    using C = T2S<TY, NT>;
    const int t = static_cast<int>(threadIdx.x);

#define at(xx, jj) node_in<LOAD>(xx, jj, G)
#define load(xx, jj, f) load_any<S, R, LOAD>(src, G, K, xx, jj, f)

    // ---- A: every Q node's step-t pre-collision values (all loads first),
    // its density to r1 and, inside P, its values to the LDS tile
    R f[C::QPER][9];
    bool ok[C::QPER];
#pragma unroll
    for (int i = 0; i < C::QPER; ++i) {
        const int q = t + i * NT;
        const int qx = q % C::QW, qy = q / C::QW;
        const NodeAt n = at(x0 - 3 + qx, j0 - 3 + qy);
        ok[i] = q < C::NQ && (LOAD == 0 || n.in);
        if (ok[i]) load(n.x, n.j, f[i]);
    }
#pragma unroll
    for (int i = 0; i < C::QPER; ++i) {
        const int q = t + i * NT;
        if (q < C::NQ) {
            const int qx = q % C::QW, qy = q / C::QW;
            r1[qy][qx] = ok[i] ? sum9(f[i]) : R(0);
            if (ok[i] && qx >= 1 && qx <= C::PW && qy >= 1 && qy <= C::PH) {
#pragma unroll
                for (int k = 0; k < 9; ++k) pb[k][qy - 1][qx - 1] = f[i][k];
            }
        }
    }
    __syncthreads();

    // ---- B: collide P in place, step-t post-collision values to the LDS tile
#pragma unroll
    for (int i = 0; i < C::PPER; ++i) {
        const int p = t + i * NT;
        const int px = p % C::PW, py = p / C::PW;
        const NodeAt n = at(x0 - 2 + px, j0 - 2 + py);
        if (p < C::NP && (LOAD == 0 || n.in)) {
            R v[9], o[9], gx, gy;
#pragma unroll
            for (int k = 0; k < 9; ++k) v[k] = pb[k][py][px];
            gradient<R, C::QW, WALLS>(r1, px + 1, py + 1, r1[py + 1][px + 1], n.x, n.j, G, K, gx,
                                      gy);
            const Pre<R> pr = collide_pre<R, DEV, COLL>(v, K);
            collide_post<R, DEV, COLL, HU>(v, pr, gx, gy, G.corr, K, o);
#pragma unroll
            for (int k = 0; k < 9; ++k) pb[k][py][px] = static_cast<R>(static_cast<S>(o[k]));
        }
    }
    __syncthreads();

    // ---- C: step-t+1 pre-collision values of the tile's rows of this thread
    // (registers) and the densities of the tile and its ring (r2 in the space
    // of r1)
    const int tx = t & (kWave - 1);
    const int tw = t >> 6;
    R g[C::RPT][9], rco[C::RPT];
#pragma unroll
    for (int r = 0; r < C::RPT; ++r) {
        const int ty = tw + r * C::WAVES;
        const NodeAt no = at(x0 + tx, j0 + ty);
        rco[r] = R(0);
        if (LOAD == 0 || no.in) {
            pull_lds<R, R, C::PW, C::PH, WALLS>(pb, tx + 2, ty + 2, no.x, no.j, G, K, g[r]);
            rco[r] = sum9(g[r]);
        }
    }
    int cx = 0, cy = 0;
    if (t < C::CW) {
        cx = t;
        cy = 0;
    } else if (t < 2 * C::CW) {
        cx = t - C::CW;
        cy = C::CH - 1;
    } else if (t < 2 * C::CW + TY) {
        cx = 0;
        cy = 1 + t - 2 * C::CW;
    } else {
        cx = C::CW - 1;
        cy = 1 + t - 2 * C::CW - TY;
    }
    const bool hasc = t < C::NCR;
    const NodeAt nc = at(x0 - 1 + cx, j0 - 1 + cy);
    R rcr = R(0);
    if (hasc && (LOAD == 0 || nc.in)) {
        R h[9];
        pull_lds<R, R, C::PW, C::PH, WALLS>(pb, cx + 1, cy + 1, nc.x, nc.j, G, K, h);
        rcr = sum9(h);
    }
    // r2 aliases r1: every read of r1 (step B) is behind the last barrier
#pragma unroll
    for (int r = 0; r < C::RPT; ++r) r2[tw + r * C::WAVES + 1][tx + 1] = rco[r];
    if (hasc) r2[cy][cx] = rcr;
    __syncthreads();

    // ---- D: collide the tile's rows of this thread, step t+1 to the
    // destination buffer
#pragma unroll
    for (int r = 0; r < C::RPT; ++r) {
        const int ty = tw + r * C::WAVES;
        const int ox = x0 + tx, oj = j0 + ty;
        const NodeAt no = at(ox, oj);
        if (ox < G.nx && oj < G.ny && (LOAD == 0 || no.in)) {
            R gx, gy, o[9];
            gradient<R, C::CW, WALLS>(r2, tx + 1, ty + 1, rco[r], no.x, no.j, G, K, gx, gy);
            const Pre<R> pr = collide_pre<R, DEV, COLL>(g[r], K);
            collide_post<R, DEV, COLL, HU>(g[r], pr, gx, gy, G.corr, K, o);
            store_node(dst, G, oj, ox, o);
        }
    }
#undef at
#undef load
}

// The staged form on one 64 x TY tile at (x0, j0), by the tile's class.
template <typename S, typename R, bool DEV, int COLL, bool HU, int TY, int NT>
__device__ __forceinline__ void tile2_staged_tile(const S *__restrict__ src, S *__restrict__ dst,
                                                  const Geometry &G, const Consts<R> &K, int x0,
                                                  int j0, R (*pb)[T2S<TY, NT>::PH][T2S<TY, NT>::PW],
                                                  R *rr) {
    using C = T2S<TY, NT>;
    R(*r1)[C::QW] = reinterpret_cast<R(*)[C::QW]>(rr);
    R(*r2)[C::CW] = reinterpret_cast<R(*)[C::CW]>(rr);
    const bool walls = G.bc[kXmin] != kPeriodic || G.bc[kYmin] != kPeriodic;
    const bool rows_in = G.buf_ok && j0 >= 4 && j0 + TY + 4 <= G.ny;
    const bool cols_in = x0 >= 4 && x0 + kWave + 4 <= G.nx;
    if (rows_in && cols_in)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 0, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in && !walls)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 1, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 1, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (walls)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 2, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 2, false>(src, dst, G, K, x0, j0, pb, r1, r2);
}

template <typename S, typename R, bool DEV, int COLL, bool HU, int TY, int NT, int WPE>
__global__ void __launch_bounds__(NT, WPE)
tile2_staged_kernel(const S *__restrict__ src, S *__restrict__ dst, const Geometry G,
                    const Consts<R> K, int ntx, int nty) {
    using C = T2S<TY, NT>;
    __shared__ R pb[9][C::PH][C::PW];
    __shared__ R rr[C::QH * C::QW];
    int b = blockIdx.x;
    const int nb = static_cast<int>(gridDim.x);
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    if (b >= ntx * nty) return;                             // padding workgroup (whole block)
    // (the tile's class is chosen here rather than through tile2_staged_tile:
    // with the kernel arguments in scalar registers that form spills fewer
    // of them)
    const int x0 = (b % ntx) * kWave, j0 = (b / ntx) * TY;
    R(*r1)[C::QW] = reinterpret_cast<R(*)[C::QW]>(rr);
    R(*r2)[C::CW] = reinterpret_cast<R(*)[C::CW]>(rr);
    const bool walls = G.bc[kXmin] != kPeriodic || G.bc[kYmin] != kPeriodic;
    const bool rows_in = G.buf_ok && j0 >= 4 && j0 + TY + 4 <= G.ny;
    const bool cols_in = x0 >= 4 && x0 + kWave + 4 <= G.nx;
    if (rows_in && cols_in)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 0, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in && !walls)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 1, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 1, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (walls)
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 2, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else
        tile2_body_staged<S, R, DEV, COLL, HU, TY, NT, 2, false>(src, dst, G, K, x0, j0, pb, r1, r2);
}

// Batched staged form: a persistent grid walks a list of 64 x TY block tiles
// of all active cases (BatchTile {case, tile column, tile row}), every case
// in pull form; case c reads buf[cur ^ flip] and writes the other buffer.
template <typename S, typename R, bool DEV, int COLL, bool HU, int TY, int NT, int WPE>
__global__ void __launch_bounds__(NT, WPE)
batch_staged_kernel(S *__restrict__ buf0, S *__restrict__ buf1,
                    const BatchTile *__restrict__ tiles, const int *__restrict__ ntiles,
                    const BatchCase *__restrict__ cases, const Geometry *__restrict__ geoms,
                    const Consts<R> *__restrict__ Ks, int flip) {
    using C = T2S<TY, NT>;
    __shared__ R pb[9][C::PH][C::PW];
    __shared__ R rr[C::QH * C::QW];
    const int n = *ntiles;
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const BatchTile td = tiles[t];
        const int c = __builtin_amdgcn_readfirstlane(td.c);
        const int tcol = __builtin_amdgcn_readfirstlane(td.seg);
        const int trow = __builtin_amdgcn_readfirstlane(td.chunk);
        const int cur = __builtin_amdgcn_readfirstlane(cases[c].cur) ^ flip;
        const long long off = cases[c].off;
        const S *src = (cur ? buf1 : buf0) + off;
        S *dst = (cur ? buf0 : buf1) + off;
        tile2_staged_tile<S, R, DEV, COLL, HU, TY, NT>(src, dst, geoms[c], Ks[c], tcol * kWave,
                                                       trow * TY, pb, rr);
        __syncthreads();  // the next tile reuses the LDS tiles
    }
}

// The register form on one 64 x TY tile at (x0, j0): interior tiles take
// the buffer loads, edge tiles the per-lane x faces or the generic loader.
template <typename S, typename R, bool DEV, int COLL, bool HU, int TY>
__device__ __forceinline__ void tile2_tile(const S *__restrict__ src, S *__restrict__ dst,
                                           const Geometry &G, const Consts<R> &K, int x0, int j0,
                                           S (*pb)[T2<TY>::PH][T2<TY>::PW], R *rr) {
    using C = T2<TY>;
    R(*r1)[C::QW] = reinterpret_cast<R(*)[C::QW]>(rr);
    R(*r2)[C::CW] = reinterpret_cast<R(*)[C::CW]>(rr);
    const bool walls = G.bc[kXmin] != kPeriodic || G.bc[kYmin] != kPeriodic;
    // every node pulled for region Q (rows j0-4 .. j0+TY+3, columns
    // x0-4 .. x0+67) inside the lattice: no wrap, no wall on any path
    const bool rows_in = G.buf_ok && j0 >= 4 && j0 + TY + 4 <= G.ny;
    const bool cols_in = x0 >= 4 && x0 + kWave + 4 <= G.nx;
    if (rows_in && cols_in)
        tile2_body<S, R, DEV, COLL, HU, TY, 0, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in && !walls)
        tile2_body<S, R, DEV, COLL, HU, TY, 1, false>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (rows_in)
        tile2_body<S, R, DEV, COLL, HU, TY, 1, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else if (walls)
        tile2_body<S, R, DEV, COLL, HU, TY, 2, true>(src, dst, G, K, x0, j0, pb, r1, r2);
    else
        tile2_body<S, R, DEV, COLL, HU, TY, 2, false>(src, dst, G, K, x0, j0, pb, r1, r2);
}

template <typename S, typename R, bool DEV, int COLL, bool HU, int TY>
__global__ void __launch_bounds__(kWave * TY)
tile2_step_kernel(const S *__restrict__ src, S *__restrict__ dst, const Geometry G,
                  const Consts<R> K, int ntx, int nty) {
    using C = T2<TY>;
    __shared__ S pb[9][C::PH][C::PW];
    __shared__ R rr[C::QH * C::QW];
    int b = blockIdx.x;
    const int nb = static_cast<int>(gridDim.x);
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    if (b >= ntx * nty) return;                             // padding workgroup (whole block)
    tile2_tile<S, R, DEV, COLL, HU, TY>(src, dst, G, K, (b % ntx) * kWave, (b / ntx) * TY, pb, rr);
}

// Batched form: a persistent grid walks a list of 64 x kBatchTileRows block
// tiles of all active cases (BatchTile {case, tile column, tile row}), every
// case in pull form; case c reads buf[cur ^ flip] and writes the other
// buffer.  The LDS tiles are reused, with a barrier between tiles.
template <typename S, typename R, bool DEV, int COLL, bool HU>
__global__ void __launch_bounds__(kWave * kBatchTileRows)
batch_tile2_kernel(S *__restrict__ buf0, S *__restrict__ buf1, const BatchTile *__restrict__ tiles,
                   const int *__restrict__ ntiles, const BatchCase *__restrict__ cases,
                   const Geometry *__restrict__ geoms, const Consts<R> *__restrict__ Ks, int flip) {
    constexpr int TY = kBatchTileRows;
    using C = T2<TY>;
    __shared__ S pb[9][C::PH][C::PW];
    __shared__ R rr[C::QH * C::QW];
    const int n = *ntiles;
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const BatchTile td = tiles[t];
        const int c = __builtin_amdgcn_readfirstlane(td.c);
        const int tcol = __builtin_amdgcn_readfirstlane(td.seg);
        const int trow = __builtin_amdgcn_readfirstlane(td.chunk);
        const int cur = __builtin_amdgcn_readfirstlane(cases[c].cur) ^ flip;
        const long long off = cases[c].off;
        const S *src = (cur ? buf1 : buf0) + off;
        S *dst = (cur ? buf0 : buf1) + off;
        tile2_tile<S, R, DEV, COLL, HU, TY>(src, dst, geoms[c], Ks[c], tcol * kWave, trow * TY, pb,
                                            rr);
        __syncthreads();  // the next tile reuses the LDS tiles
    }
}

// Rows of the register form's output tile.  Measured on the 2048 x 8192
// lattice (FP32 storage and arithmetic, per pair of steps): 64 x 16 tiles
// (1024 threads, one workgroup per CU by its registers) 442 us, the same
// with the compiler held to two workgroups per CU 351 us, 64 x 8 tiles (512
// threads, three workgroups per CU) 341 us.  FP64 takes 64 x 8 too: its
// step-t tile in LDS (67 KB) leaves room for two workgroups per CU, and a
// taller staged tile in FP64 would leave room for one.
template <typename R>
constexpr int tile2_rows() { return 8; }

// Tile of the staged form with FP32 storage and arithmetic: rows, threads
// and the waves per SIMD asked of the compiler (0 rows: the register form
// for every type).  Measured on the same lattice, per pair of steps, with
// the same collision code (two runs; 64 x 16, timed in both, gave 309-311
// us in each): 64 x 8 register form 336-338 us; staged 64 x 12 / 384
// threads 346, 64 x 14 / 448 328, 64 x 16 / 512 309-311, 64 x 18 / 576 467,
// 64 x 20 / 640 439, 64 x 24 / 768 285 (77 KB of LDS, two workgroups per
// CU), 64 x 32 / 1024 380 (one workgroup per CU).
constexpr int kStagedRows = 24, kStagedThreads = 768, kStagedWaves = 6;

// The automatic choice takes the staged form from this many of its
// workgroups up (two per CU).  Its fixed cost per launch is higher (7-8 us
// per step on lattices of up to 256 x 512 nodes, against 5-5.5 us), so
// smaller lattices run the register form: measured per step with cavity
// boundaries, register / staged, 512 x 1024 (344 staged workgroups) 9.64 /
// 9.72 us, 1024 x 1024 (688) 13.46 / 12.95, 1024 x 2048 21.84 / 19.51,
// 2048 x 4096 88.30 / 76.67.
constexpr int kStagedMinGroups = 512;

int staged_groups(const Geometry &G) {
    return ((G.nx + kWave - 1) / kWave) * ((G.ny + kStagedRows - 1) / kStagedRows);
}

template <typename S, typename R, bool DEV>
hipError_t staged_dispatch(int coll, bool hu, const S *s, S *d, const Geometry &G,
                           const Consts<R> &K, hipStream_t st) {
    constexpr int TY = kStagedRows, NT = kStagedThreads, WPE = kStagedWaves;
    const int ntx = (G.nx + kWave - 1) / kWave, nty = (G.ny + TY - 1) / TY;
    const int n = ntx * nty;
    const dim3 grid((n + 7) / 8 * 8), block(NT);
#define LBM_T2S(CO, H) \
    hipLaunchKernelGGL((tile2_staged_kernel<S, R, DEV, CO, H, TY, NT, WPE>), grid, block, 0, st, s, d, G, K, ntx, nty)
    if (coll == kRC) {
        if (hu) LBM_T2S(kRC, true); else LBM_T2S(kRC, false);
    } else {
        if (hu) LBM_T2S(kRNR, true); else LBM_T2S(kRNR, false);
    }
#undef LBM_T2S
    return hipGetLastError();
}

template <typename S, typename R, bool DEV>
hipError_t tile2_dispatch(int coll, bool hu, int form, const void *src, void *dst,
                          const Geometry &G, const Consts<R> &K, hipStream_t st) {
    const S *s = static_cast<const S *>(src);
    S *d = static_cast<S *>(dst);
    if constexpr (sizeof(R) == 4 && sizeof(S) == 4) {
        if (form == kFormStaged) return staged_dispatch<S, R, DEV>(coll, hu, s, d, G, K, st);
    }
    if (form == kFormStaged) return hipErrorInvalidValue;
    constexpr int TY = tile2_rows<R>();
    const int ntx = (G.nx + kWave - 1) / kWave, nty = (G.ny + TY - 1) / TY;
    const int n = ntx * nty;
    const dim3 grid((n + 7) / 8 * 8), block(kWave * TY);
#define LBM_T2(CO, H) \
    hipLaunchKernelGGL((tile2_step_kernel<S, R, DEV, CO, H, TY>), grid, block, 0, st, s, d, G, K, ntx, nty)
    if (coll == kRC) {
        if (hu) LBM_T2(kRC, true); else LBM_T2(kRC, false);
    } else {
        if (hu) LBM_T2(kRNR, true); else LBM_T2(kRNR, false);
    }
#undef LBM_T2
    return hipGetLastError();
}

}  // namespace

int two_step_form(int prec, int form, const Geometry &G) {
    if (prec != kFP32Dev) return kFormRegister;  // the staged form is FP32 only
    if (form != kFormAuto) return form;
    return staged_groups(G) >= kStagedMinGroups ? kFormStaged : kFormRegister;
}

hipError_t launch_step2(int prec, int coll, bool hu, int form, const void *src, void *dst,
                        const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                        hipStream_t st) {
    if (form == kFormStaged && prec != kFP32Dev) return hipErrorInvalidValue;
    const int f = two_step_form(prec, form, G);
    switch (prec) {
    case kFP64: return tile2_dispatch<double, double, false>(coll, hu, f, src, dst, G, Kd, st);
    case kFP32Dev: return tile2_dispatch<float, float, true>(coll, hu, f, src, dst, G, Kf, st);
    case kFP64Dev: return tile2_dispatch<double, double, true>(coll, hu, f, src, dst, G, Kd, st);
    case kFP32DevF64: return tile2_dispatch<float, double, true>(coll, hu, f, src, dst, G, Kd, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename S, typename R, bool DEV>
static hipError_t batch_tile2_dispatch(int coll, bool hu, void *b0, void *b1,
                                       const BatchTile *tiles, const int *ntiles,
                                       const BatchCase *cases, const Geometry *geoms,
                                       const Consts<R> *K, int flip, int wgs, hipStream_t st) {
    static_assert(kBatchTileRows == tile2_rows<R>(), "block tiles of the register form");
    const dim3 grid(wgs), block(kWave * kBatchTileRows);
#define LBM_BT2(CO, H)                                                                            \
    hipLaunchKernelGGL((batch_tile2_kernel<S, R, DEV, CO, H>), grid, block, 0, st,                 \
                       static_cast<S *>(b0), static_cast<S *>(b1), tiles, ntiles, cases, geoms,   \
                       K, flip)
    if (coll == kRC) {
        if (hu) LBM_BT2(kRC, true); else LBM_BT2(kRC, false);
    } else {
        if (hu) LBM_BT2(kRNR, true); else LBM_BT2(kRNR, false);
    }
#undef LBM_BT2
    return hipGetLastError();
}

hipError_t launch_batch_staged(int prec, int coll, bool hu, void *b0, void *b1,
                               const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                               const Geometry *geoms, const Consts<float> *Kf, int flip, int wgs,
                               hipStream_t st) {
    if (prec != kFP32Dev) return hipErrorInvalidValue;  // the staged form is FP32 only
    static_assert(kBatchStagedRows == kStagedRows, "block tiles of the staged form");
    constexpr int TY = kStagedRows, NT = kStagedThreads, WPE = kStagedWaves;
    const dim3 grid(wgs), block(NT);
    float *s0 = static_cast<float *>(b0), *s1 = static_cast<float *>(b1);
#define LBM_BST(CO, H)                                                                             \
    hipLaunchKernelGGL((batch_staged_kernel<float, float, true, CO, H, TY, NT, WPE>), grid, block, \
                       0, st, s0, s1, tiles, ntiles, cases, geoms, Kf, flip)
    if (coll == kRC) {
        if (hu) LBM_BST(kRC, true); else LBM_BST(kRC, false);
    } else {
        if (hu) LBM_BST(kRNR, true); else LBM_BST(kRNR, false);
    }
#undef LBM_BST
    return hipGetLastError();
}

hipError_t launch_batch_tile2(int prec, int coll, bool hu, void *b0, void *b1,
                              const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                              const Geometry *geoms, const Consts<double> *Kd,
                              const Consts<float> *Kf, int flip, int wgs, hipStream_t st) {
    switch (prec) {
    case kFP64: return batch_tile2_dispatch<double, double, false>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, wgs, st);
    case kFP32Dev: return batch_tile2_dispatch<float, float, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kf, flip, wgs, st);
    case kFP64Dev: return batch_tile2_dispatch<double, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, wgs, st);
    case kFP32DevF64: return batch_tile2_dispatch<float, double, true>(coll, hu, b0, b1, tiles, ntiles, cases, geoms, Kd, flip, wgs, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
