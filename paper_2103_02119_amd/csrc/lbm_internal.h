// Internal declarations shared by the HIP kernels and the host side of the
// C ABI (include/lbm.h).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kWavesPerBlock = 4;   // independent wavefronts per workgroup
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxRows = 64;        // rows marched by one wavefront (halo pass width)
constexpr int kReduceBlock = 256;
constexpr int kMaxPartials = 4096;  // per-block partial sums of the reductions

enum Prec { kFP64 = 0, kFP32Dev = 1, kFP64Dev = 2, kFP32DevF64 = 3 };
// populations stored as FP32 deviations (kFP32Dev, kFP32DevF64)
__host__ __device__ constexpr bool f32_storage(int prec) { return prec == kFP32Dev || prec == kFP32DevF64; }
enum Face { kXmin = 0, kXmax = 1, kYmin = 2, kYmax = 3 };
enum Bc { kPeriodic = 0, kWall = 1, kMovingWall = 2 };
enum Coll { kRC = 0, kRNR = 1 };

// (cx, cy) of direction k in the ordering of Eq. 2; e = (cx, a cy).
__host__ __device__ constexpr int cx_of(int k) {
    return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int k) {
    return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int k) {
    return k == 0 ? 0 : k == 1 ? 3 : k == 2 ? 4 : k == 3 ? 1 : k == 4 ? 2
         : k == 5 ? 7 : k == 6 ? 8 : k == 7 ? 5 : 6;
}

// Lattice geometry and launch tiling (uniform kernel argument).
struct Geometry {
    int nx, ny, pitch;       // pitch: row stride in values (multiple of 64)
    int nseg;                // 64-column segments per row
    int rows;                // rows marched by one wavefront
    int nchunk;              // row chunks
    int ntile;               // nseg * nchunk wavefront tiles
    int nblocks;             // workgroups of the step kernel
    int xcd_remap;           // 1: contiguous tiles per XCD (nblocks % 8 == 0)
    int bc[4];               // Bc per face
    int corr;                // 1: Eq. 23-27 corrections on
    int buf_ok;              // 1: a population buffer is below 4 GiB (buffer addressing)
    int nt_store;            // 1: non-temporal population stores (buffers exceed the MALL)
    int tile_rows;           // > 0: the one-node-per-thread tile kernel with tiles of 64 x
                             // tile_rows (taken when no obstacle mask is set); 0: the march
    long long plane;         // pitch * ny
    const unsigned char *mask;        // obstacle mask [ny][pitch], nonzero = solid (or null)
    const unsigned char *tile_solid;  // per step-kernel tile: a solid node in its neighbourhood
};

// Model constants in the arithmetic type R of a kernel.
template <typename R>
struct Consts {
    R a, inv_a, a2, inv_a2, half_inv_a;
    R s, s2;                 // cs2, cs2^2
    R rr;                    // deviation origin rho0 (0 when f itself is stored)
    R Fx, Fy, hFx, hFy;      // force and half force
    R w[9];                  // omega_j
    R om[9];                 // 1 - omega_j
    R sw[9];                 // 1 - omega_j / 2
    R k3, k4;                // 1/omega_3 - 1/2, 1/omega_4 - 1/2
    R b1c, b2c, c1c, c2c;    // u-independent parts of B1/rho, B2/rho, C1/rho, C2/rho (Eq. 40)
    R e1, e2;                // (3 cs2 - 1)/2, (3 cs2 - a^2)/2 (B3/ux, B4/uy of Eq. 40)
    R q1, q2;                // 1 - 3 cs2, a^2 - 3 cs2 (Eq. 23-24)
    R dwall[4][9];           // (feq_opp(k) - feq_k)(rho0, u_wall[face]) per face
    R rest[9];               // stored value of the rest state (solid nodes): rho0 w_k, or 0 as a deviation
};

// Per-context constants for the conversion kernels (always FP64).
struct HostSide {
    double wrest[9];         // rest weights w_k = feq_k(1, 0)
    double rho0, a, s, Fx, Fy;
    int dev;                 // 1: storage holds f - w rho0
};

// ---- batches of independent lattices (one launch advances all of them) ----
// The two ping-pong buffers of a batch are two allocations with the same
// layout; case c occupies values off .. off + 9 plane of each.
struct BatchCase {
    long long off;           // first value of the case in either buffer
    int cur;                 // buffer (0 / 1) holding the current state
    int pull;                // 1: the current buffer holds post-collision values (pull form)
};
// Work item of the batched step: a 64-column x rows tile of one case.
struct BatchTile {
    int c, seg, chunk, pad;
};
// Work item of the batched reductions: nodes [start, start + count) of case c,
// whose current / previous buffers are in pull form when pc / pp is set.
struct BatchRed {
    int c, start, count, flags;  // flags: bit 0 pc, bit 1 pp
};
constexpr int kBatchRedNodes = 4096;  // nodes per reduction work item
constexpr int kBatchTileRows = 8;     // rows of a block tile of the batched tile kernel
constexpr int kBatchStagedRows = 24;  // rows of a block tile of the batched staged two-step kernel

// ---- host helpers shared by the single-lattice and batch front ends ----
// (implemented in lbm_api.hip; the lbm.h types are opaque here)
struct CaseSpec {
    int nx, ny;
    double a;
    double rates[9];
    lbm_bc bc;
    double cs2, force[2], rho0;
    int prec, corr;
};
int validate_case(int nx, int ny, double r, const double *rates, const lbm_bc *bc,
                  const lbm_opts *o);  // fills the create error text on failure
void make_spec(int nx, int ny, double r, const double *rates, const lbm_bc *bc, const lbm_opts *o,
               CaseSpec &spec);
template <typename R>
void fill_consts(const CaseSpec &c, Consts<R> &K);
void fill_host_side(const CaseSpec &c, HostSide &H);
void base_geometry(const CaseSpec &c, size_t f_bytes, Geometry &G);
void set_rows(Geometry &G, int rows);  // rows per wavefront and the tile counts that follow
// 1 if a solid node lies within two nodes of step tile (seg, chunk): rows
// j0 - 2 .. j1 + 1, columns x0 - 2 .. x0 + 65 (wrapped where periodic) -- the
// tile pulls from one node around it, and the ring / halo densities it forms
// pull from one node further out
int tile_has_solid(const Geometry &G, const unsigned char *host_mask, int seg, int chunk);
int auto_rows(long long nodes, int prec);
int pitch_of(int nx);
const char *create_error_text();
int set_create_error(const char *msg);

// ---- launchers implemented in the kernel sources (return hipError_t) ----
// workgroups of the tile kernel for a lattice (whole groups of 8)
int tile_workgroups(const Geometry &G);
// the step kernel a launch takes: the tile kernel unless tile_rows is 0 or a mask is set
inline bool uses_tile_kernel(const Geometry &G) { return G.tile_rows > 0 && !G.mask; }
hipError_t launch_step(int prec, int coll, bool pull, bool higher_unit, const void *src, void *dst,
                       const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                       hipStream_t st);
// the march step kernel (lbm_march.hip); launch_step takes it when the tile
// kernel does not apply
hipError_t launch_march_step(int prec, int coll, bool pull, bool higher_unit, const void *src,
                             void *dst, const Geometry &G, const Consts<double> &Kd,
                             const Consts<float> &Kf, hipStream_t st);
// two steps per launch (lbm_tile2.hip): src must hold post-collision values
// (pull form) and the lattice no obstacle mask; dst receives step t+1.
// form: kFormAuto, kFormRegister or kFormStaged (FP32 storage and arithmetic
// only); two_step_form tells which one a launch takes.
constexpr int kFormAuto = 0, kFormRegister = 1, kFormStaged = 2;
int two_step_form(int prec, int form, const Geometry &G);
hipError_t launch_step2(int prec, int coll, bool higher_unit, int form, const void *src, void *dst,
                        const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                        hipStream_t st);
// streaming copy of n16 16-byte words (the measured bandwidth ceiling);
// workgroups <= 0 selects the default grid
hipError_t launch_stream_copy(void *dst, const void *src, long long n16, int workgroups,
                              hipStream_t st);
// workgroups (= partial sums) of the reductions on a lattice (<= kMaxPartials)
int reduce_partials(const Geometry &G);
hipError_t launch_init_feq(int prec, void *dst, const double *rho, const double *ux,
                           const double *uy, const Geometry &G, const HostSide &H, hipStream_t st);
hipError_t launch_set_populations(int prec, void *dst, const double *f, const Geometry &G,
                                  const HostSide &H, hipStream_t st);
// pull: 1 if the buffer holds post-collision values of the previous step
hipError_t launch_get_populations(int prec, bool pull, const void *src, double *f,
                                  const Geometry &G, const Consts<double> &Kd,
                                  const Consts<float> &Kf, const HostSide &H, hipStream_t st);
// f[9][n] (FP64, full populations) = mean of the states in cur and prev
hipError_t launch_average_states(int prec, bool pull_cur, const void *cur, bool pull_prev,
                                 const void *prev, double *f, const Geometry &G,
                                 const Consts<double> &Kd, const HostSide &H, hipStream_t st);
hipError_t launch_moments(int prec, bool pull, const void *src, double *rho, double *ux,
                          double *uy, const Geometry &G, const Consts<double> &Kd,
                          const Consts<float> &Kf, const HostSide &H, hipStream_t st);
// local viscous stress from the state in src and its densities rho[ny][nx]
hipError_t launch_stress(int prec, bool pull, const void *src, const double *rho, double *sxx,
                         double *syy, double *sxy, const Geometry &G, const Consts<double> &Kd,
                         const HostSide &H, hipStream_t st);
// out[0..2] = sum rho, sum rho ux, sum rho uy, out[3] = 1 if NaN/Inf met
hipError_t launch_sums(int prec, bool pull, const void *src, double *partials, double *out,
                       const Geometry &G, const Consts<double> &Kd, const Consts<float> &Kf,
                       const HostSide &H, hipStream_t st);
// batched step over the tile list (count in *ntiles, device memory) on a
// persistent grid of `workgroups`; case c reads buf[cur ^ flip] and is in pull
// form when force_pull or its own flag says so
hipError_t launch_batch_step(int prec, int coll, bool higher_unit, void *buf0, void *buf1,
                             const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                             const Geometry *geoms,
                             const Consts<double> *Kd, const Consts<float> *Kf, int flip,
                             int force_pull, int workgroups, hipStream_t st);
// batched tile kernel over a list of 64 x kBatchTileRows block tiles
// (BatchTile {case, tile column, tile row}) on a persistent grid of `workgroups`
hipError_t launch_batch_tile(int prec, int coll, bool higher_unit, void *buf0, void *buf1,
                             const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                             const Geometry *geoms, const Consts<double> *Kd,
                             const Consts<float> *Kf, int flip, int force_pull, int workgroups,
                             hipStream_t st);
// two steps per launch over the same block tiles (lbm_tile2.hip): every
// active case must be in pull form and without a mask
hipError_t launch_batch_tile2(int prec, int coll, bool higher_unit, void *buf0, void *buf1,
                              const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                              const Geometry *geoms, const Consts<double> *Kd,
                              const Consts<float> *Kf, int flip, int workgroups, hipStream_t st);
// the staged two-step form over a list of 64 x kBatchStagedRows block tiles
// (LBM_FP32_DEV only)
hipError_t launch_batch_staged(int prec, int coll, bool higher_unit, void *buf0, void *buf1,
                               const BatchTile *tiles, const int *ntiles, const BatchCase *cases,
                               const Geometry *geoms, const Consts<float> *Kf, int flip,
                               int workgroups, hipStream_t st);
// per-case residual sums of the batch: out[4 c + 0..3] as for launch_residual,
// over the cases named by the reduction items (items of a case are contiguous)
hipError_t launch_batch_residual(int prec, const void *buf0, const void *buf1,
                                 const BatchRed *items, int nitems,
                                 const BatchCase *cases, const Geometry *geoms,
                                 const Consts<double> *Kd, const HostSide *H, double *partials,
                                 const int *case_first, const int *case_count, int ncases,
                                 double *out, hipStream_t st);
// out[0] = sum |u_cur - u_prev|^2, out[1] = sum |u_cur|^2, out[3] = NaN/Inf flag
hipError_t launch_residual(int prec, bool pull_cur, const void *cur, bool pull_prev,
                           const void *prev, double *partials, double *out, const Geometry &G,
                           const Consts<double> &Kd, const Consts<float> &Kf, const HostSide &H,
                           hipStream_t st);
// out[0..3] as launch_residual and out[4..7] as launch_sums (of cur), in one
// pass; partials holds 8 values per block (8 * kMaxPartials)
hipError_t launch_check(int prec, bool pull_cur, const void *cur, bool pull_prev,
                        const void *prev, double *partials, double *out, const Geometry &G,
                        const Consts<double> &Kd, const Consts<float> &Kf, const HostSide &H,
                        hipStream_t st);

}  // namespace lbm
