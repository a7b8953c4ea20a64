// The tile step kernel: one node per thread, a workgroup of TY wavefronts
// owning a 64 x TY tile with the density ring in LDS (the default step when
// no obstacle mask is set), and its batched form.
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

// ------------------------------------------------------------ tile kernel


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
static hipError_t tile_dispatch(int coll, bool pull, bool hu, const void *src, void *dst,
                                const Geometry &G, const Consts<R> &K, hipStream_t st) {
    const S *s = static_cast<const S *>(src);
    S *d = static_cast<S *>(dst);
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

hipError_t launch_step(int prec, int coll, bool pull, bool hu, const void *src, void *dst,
                       const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                       hipStream_t st) {
    if (!uses_tile_kernel(G)) return launch_march_step(prec, coll, pull, hu, src, dst, G, Kd, Kf, st);
    switch (prec) {
    case kFP64: return tile_dispatch<double, double, false>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32Dev: return tile_dispatch<float, float, true>(coll, pull, hu, src, dst, G, Kf, st);
    case kFP64Dev: return tile_dispatch<double, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    case kFP32DevF64: return tile_dispatch<float, double, true>(coll, pull, hu, src, dst, G, Kd, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
