// The march step kernel (one wavefront marches 64 columns x `rows` rows,
// keeping a window of rows in registers), used for an explicit rows-per-
// wavefront choice, for lattices with an obstacle mask and by the batch.
//   * The density gradient (the only non-local input of the collision,
//     Sec. 2.3) needs rho of the 4 neighbours at the same time level: the row
//     below and above come from the marching window, the left/right
//     neighbours from a wavefront shuffle, and the two columns beyond the
//     segment from a halo pass done once per wavefront (one halo node per
//     lane).
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

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

template <typename S, typename R, bool DEV>
static hipError_t march_dispatch(int coll, bool pull, bool hu, const void *src, void *dst,
                                 const Geometry &G, const Consts<R> &K, hipStream_t st) {
    const dim3 grid(G.nblocks), block(kBlock);
    const S *s = static_cast<const S *>(src);
    S *d = static_cast<S *>(dst);
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

hipError_t launch_march_step(int prec, int coll, bool pull, bool hu, const void *src, void *dst,
                             const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                             hipStream_t st) {
    switch (prec) {
    case kFP64: return march_dispatch<double, double, false>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32Dev: return march_dispatch<float, float, true>(coll, pull, hu, src, dst, G, Kf, st);
    case kFP64Dev: return march_dispatch<double, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32DevF64: return march_dispatch<float, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
