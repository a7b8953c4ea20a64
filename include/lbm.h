/*
 * lbm.h -- C ABI of the MI355X library for the rectangular-lattice central
 * moment lattice Boltzmann method of E. Yahia & K. N. Premnath, "Central
 * Moment Lattice Boltzmann Method on a Rectangular Lattice" (arXiv
 * 2103.02119).
 *
 * The library advances a D2Q9 lattice with grid aspect ratio a = dy/dx
 * (Sec. 2.1) by the fused collide-and-stream step:
 *   - RC-LBM (Sec. 4): relaxation of central moments toward the Maxwell-matched
 *     central equilibria of Eq. 49, including the isotropy and Galilean
 *     invariance corrections of Eq. 23-27 with the local strain rate of
 *     Eq. 37-38 (the default);
 *   - RNR-LBM (Sec. 3): the raw-moment special case;
 *   - perfect-shift streaming with periodic faces, half-way bounce-back walls
 *     and moving walls (Sec. 5.2, Eq. 57-59);
 *   - the macroscopic fields rho = sum f, rho u = sum f e + F/2.
 * Every step runs in hand-written HIP kernels for gfx950 on the caller's
 * stream.  There is no CPU fallback: without a usable GPU every call that
 * needs the device returns LBM_E_DEVICE.
 *
 * Conventions
 *   - Lattice units: dx = dt = 1, dy = a; e_i = (cx_i, a cy_i) with the
 *     ordering of Eq. 2: 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1),
 *     5 (1,1), 6 (-1,1), 7 (-1,-1), 8 (1,-1) in (cx, cy).
 *   - Node (i, j), 0 <= i < nx, 0 <= j < ny, sits at x = i, y = j a; a wall
 *     lies half a node beyond the first/last row or column.
 *   - Host scalar fields are double[ny][nx]; host populations are
 *     double[9][ny][nx]; x fastest, C order.
 *   - All functions return an int status (LBM_OK = 0, negative = error); no
 *     exception or signal crosses the ABI.  lbm_last_error() describes the
 *     last failure of a context.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,    /* invalid argument; nothing was changed */
    LBM_E_NOMEM = -2,    /* a device or host allocation failed */
    LBM_E_DEVICE = -3,   /* a HIP call failed or no GPU is usable */
    LBM_E_UNSTABLE = -4, /* a reduction met NaN or Inf (the run has blown up) */
    LBM_E_STATE = -5     /* the call needs a state the context is not in */
};

/* boundary type of a face */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1, LBM_BC_MOVING_WALL = 2 };
/* face index into lbm_bc */
enum { LBM_FACE_XMIN = 0, LBM_FACE_XMAX = 1, LBM_FACE_YMIN = 2, LBM_FACE_YMAX = 3 };
/* collision model */
enum { LBM_RC = 0, LBM_RNR = 1 };
/* storage and arithmetic precision:
 *   LBM_FP64      populations f stored and collided in FP64;
 *   LBM_FP32_DEV  deviations g = f - w rho0 stored and collided in FP32
 *                 (w = rest-state equilibrium weights); reductions in FP64;
 *   LBM_FP64_DEV  the deviation algorithm in FP64 (a check of that algebra);
 *   LBM_FP32_DEV_F64  deviations stored in FP32 (FP32 traffic), collided in FP64
 *                 (FP64 vector arithmetic runs at the unpacked FP32 rate on CDNA). */
enum { LBM_FP64 = 0, LBM_FP32_DEV = 1, LBM_FP64_DEV = 2, LBM_FP32_DEV_F64 = 3 };

/* Boundary description.  x-min/x-max must both be periodic or both not; the
 * same for y-min/y-max.  u_wall[face] = (Ux, Uy) is used by
 * LBM_BC_MOVING_WALL faces (Sec. 5.2: f_i = f~_ibar - (feq_ibar - feq_i)(rho_w, u_w),
 * rho_w = rho0).  A link that crosses two faces (a corner) uses the moving
 * face if exactly one of them moves, else the y face. */
typedef struct {
    int type[4];
    double u_wall[4][2];
} lbm_bc;

typedef struct {
    double cs2;        /* squared speed of sound, 0 < cs2 < min(1, a^2) (rest weights
                          positive); 0 selects min(1/3, 0.64 a^2) */
    double force[2];   /* uniform body force (Fx, Fy), lattice units (Eq. 13) */
    double rho0;       /* reference density: wall density and deviation origin; 0 => 1 */
    int collision;     /* LBM_RC (default) or LBM_RNR */
    int precision;     /* LBM_FP64 (default), LBM_FP32_DEV, LBM_FP64_DEV, LBM_FP32_DEV_F64 */
    int corrections;   /* 1 (default): Eq. 23-27 corrections; 0: leave them out */
    int rows_per_wave; /* launch shape override (rows marched by one wavefront);
                          0 = automatic */
    void *stream;      /* hipStream_t the library enqueues on; NULL = null stream */
    void *f_a, *f_b;   /* optional caller-owned device buffers of f_bytes each
                          (lbm_required_bytes); NULL => the library allocates */
    size_t f_bytes;
} lbm_opts;

typedef struct lbm_ctx lbm_ctx;

/* Fills *o with the defaults listed above. */
void lbm_default_opts(lbm_opts *o);

/* Device bytes of one population buffer (9 planes of ny rows, each row padded
 * to a multiple of 64 values) for the given precision.
 * Errors: LBM_E_INVAL for nx or ny < 3, a bad precision or a lattice whose
 * plane (one population, padded rows) exceeds 4 GiB. */
int lbm_required_bytes(int nx, int ny, int precision, size_t *f_bytes);

/* Creates a lattice of nx x ny nodes with aspect ratio r = a = dy/dx
 * (Sec. 2.1) and relaxation rates rates[0..8] = omega_0..omega_8 (Eq. 5-6;
 * the paper uses omega_4 = omega_5 = 1/tau, all others 1, with
 * nu = cs2 (1/omega_4 - 1/2) and zeta = cs2 (1/omega_3 - 1/2), Eq. 32-33).
 * The populations start at the rest equilibrium f = feq(rho0, 0).
 * opts may be NULL (defaults).  Caller-owned buffers are borrowed, never
 * freed, and must outlive the context.  Enqueues work on the stream and
 * returns without waiting.
 * Errors: LBM_E_INVAL when nx or ny < 3, r <= 0, cs2 not in (0, min(1, r^2)),
 * an omega not in (0, 2), mismatched periodic faces, an unknown enum value or
 * a caller buffer smaller than lbm_required_bytes; LBM_E_DEVICE without a
 * usable GPU; LBM_E_NOMEM when allocation fails.  *out is NULL on error. */
int lbm_create(int nx, int ny, double r, const double rates[9], const lbm_bc *bc,
               const lbm_opts *opts, lbm_ctx **out);

/* Sets f = feq(rho, u) at every node (product form of T^{-1} F(-u) applied to
 * Eq. 49 without corrections; no non-equilibrium part).  rho, ux, uy are host
 * double[ny][nx]; NULL means rho0 (rho) or 0 (ux, uy).  Synchronizes the
 * stream.  Errors: LBM_E_DEVICE. */
int lbm_set_fields(lbm_ctx *ctx, const double *rho, const double *ux, const double *uy);

/* Enqueues n >= 0 collide-and-stream steps on the stream (Sec. 3 / Sec. 4
 * algorithm: pull streaming, macroscopic fields, collision; each launch
 * fuses one step, or two steps with the intermediate state kept on chip, see
 * lbm_set_steps_per_launch) and returns without waiting.  Under the automatic
 * choice the call's last launch advances one step, so lbm_residual of the
 * last step is always available afterwards.
 * Errors: LBM_E_INVAL for n < 0; LBM_E_DEVICE if a launch fails. */
int lbm_step(lbm_ctx *ctx, long n);

/* Steps fused into one launch by later lbm_step calls: 1, 2 or 0 (automatic,
 * the default).  Two steps per launch (temporal blocking) read the state of
 * step t-1 once, keep each tile's step-t state in on-chip memory and write
 * step t+1, halving the population traffic per step; results are bit-identical
 * to one step per launch.  They apply only without an obstacle mask (with a
 * mask every launch advances one step).  Automatic: two on every lattice
 * without a mask (measured faster from 64 x 32 nodes up).  With
 * an explicit 2 an lbm_step call advances pairs of steps while two remain, so
 * after an even count the state one step back is not held and lbm_residual /
 * lbm_check_async / lbm_check_into return LBM_E_STATE until a one-step launch
 * (an odd count, or lbm_step(ctx, 1)).
 * Errors: LBM_E_INVAL (ctx NULL, k not 0, 1 or 2). */
int lbm_set_steps_per_launch(lbm_ctx *ctx, int k);

/* Steps per launch that lbm_step currently takes for a long run (1 or 2),
 * after the automatic choice and the mask rule; LBM_E_INVAL for a NULL ctx. */
int lbm_steps_per_launch(const lbm_ctx *ctx);

/* Form of the two-steps-per-launch kernel, a tuning choice with no effect on
 * the results (both are bit-identical to one step per launch):
 *   LBM_FORM_REGISTER  64 x 8 node tiles, the step-t values of a thread's
 *                      nodes held in registers between phases;
 *   LBM_FORM_STAGED    64 x 24 node tiles with every step-t value staged in
 *                      on-chip memory, which recomputes fewer halo nodes
 *                      (1.12 collisions per lattice update against 1.30);
 *                      LBM_FP32_DEV only;
 *   LBM_FORM_AUTO      (the default) staged for LBM_FP32_DEV once it has at
 *                      least 512 tiles, else register.
 * Errors: LBM_E_INVAL (ctx NULL, an unknown form, LBM_FORM_STAGED with a
 * precision other than LBM_FP32_DEV). */
enum { LBM_FORM_AUTO = 0, LBM_FORM_REGISTER = 1, LBM_FORM_STAGED = 2 };
int lbm_set_two_step_form(lbm_ctx *ctx, int form);

/* The form the next two-step launch takes (LBM_FORM_REGISTER or
 * LBM_FORM_STAGED), after the automatic choice; LBM_E_INVAL for a NULL ctx. */
int lbm_two_step_form(const lbm_ctx *ctx);

/* Macroscopic fields at the current time level: rho = sum f,
 * u = (sum f e + F/2) / rho (Sec. 3, "update hydrodynamic fields"), written
 * to host double[ny][nx] arrays; any pointer may be NULL.  Synchronizes.
 * Errors: LBM_E_DEVICE. */
int lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy);

/* Steady-state residual of the last step,
 * R = sqrt(sum |u^n - u^{n-1}|^2) / sqrt(sum |u^n|^2), summed in FP64 over all
 * fluid nodes with a deterministic two-pass reduction.  Synchronizes.
 * Errors: LBM_E_STATE before the first step (or after set_fields /
 * set_populations, or when the last launch advanced two steps under an
 * explicit lbm_set_steps_per_launch(ctx, 2)); LBM_E_UNSTABLE if any velocity
 * is NaN or Inf (*R is then NaN); LBM_E_DEVICE. */
int lbm_residual(lbm_ctx *ctx, double *R);

/* Local viscous stress at the current time level, computed in FP64 from the
 * populations alone (no finite differences of the velocity): the strain
 * rate d_x u_x, d_y u_y of Eq. 37-38 from the second-order non-equilibrium
 * moments m_3, m_4 with the density-gradient terms of Eq. 40 (central
 * differences, neighbours across walls or on solid nodes replaced by the node
 * itself, as in the collision), the shear rate d_y u_x + d_x u_y from m_5
 * (Eq. 39, no correction by Eq. 27), then the viscous stress of Eq. 30-31:
 * sxx = rho [nu (2 d_x u_x - div u) + zeta div u], syy likewise,
 * sxy = rho nu' (d_y u_x + d_x u_y), nu from omega_4, nu' from omega_5
 * (Eq. 32), zeta from omega_3 (Eq. 33).  Host double[ny][nx] arrays; any
 * pointer may be NULL; solid nodes get 0.  Synchronizes.
 * Errors: LBM_E_INVAL (ctx NULL), LBM_E_NOMEM (staging buffer), LBM_E_DEVICE. */
int lbm_stress(lbm_ctx *ctx, double *sxx, double *syy, double *sxy);

/* FP64 totals over all fluid nodes at the current time level: out[0] = sum rho,
 * out[1] = sum rho ux, out[2] = sum rho uy (momentum including the F/2
 * shift).  Deterministic.  Synchronizes.  Errors: LBM_E_UNSTABLE (NaN/Inf),
 * LBM_E_DEVICE. */
int lbm_sums(lbm_ctx *ctx, double out[3]);

/* lbm_residual and lbm_sums of the current time level without a host wait,
 * for monitoring a run while it runs: check_async enqueues both reductions
 * and a copy of their results to pinned host memory the context owns, and
 * returns; check_result waits only for the latest enqueued check (the steps
 * enqueued after it keep the GPU busy) and returns R, sums[0..2] and the step
 * count at which it was taken.  A later check_async replaces the pending one;
 * one that fails leaves none pending.
 * R, sums and step may be NULL.
 * Errors: check_async: LBM_E_STATE before the first step (as lbm_residual),
 * LBM_E_NOMEM (pinned buffer), LBM_E_DEVICE.  check_result: LBM_E_STATE if no
 * check was enqueued; LBM_E_UNSTABLE if a density or velocity was NaN or Inf
 * (*R is then NaN; *step names the check); LBM_E_DEVICE. */
int lbm_check_async(lbm_ctx *ctx);
int lbm_check_result(lbm_ctx *ctx, double *R, double sums[3], long *step);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_check_async's fused
 * residual-and-sums pass with its per-workgroup partial sums in a static
 * device array of the library (at most 4096 workgroups x 8 FP64 values,
 * 256 KiB, one per GPU, held until the process ends) and its results written
 * to out, caller-owned device memory of 8 doubles:
 *   out[0] = sum |u^n - u^{n-1}|^2, out[1] = sum |u^n|^2 (R = sqrt(out[0]) /
 *   sqrt(out[1])), out[2] = 0, out[3] != 0 if a velocity was NaN or Inf;
 *   out[4..6] = sum rho, sum rho ux, sum rho uy (as lbm_sums),
 *   out[7] != 0 if a density or velocity was NaN or Inf.
 * Enqueues on the context's stream and returns without waiting; calls no
 * allocating routine.  Every call on one GPU shares its array: calls that
 * overlap on one GPU (other streams, other host threads) race, so order them
 * on one stream.  The reduction size is bounded by construction; a lattice
 * needing more partials than the array holds is rejected with LBM_E_INVAL.
 * Errors: LBM_E_INVAL (NULL argument), LBM_E_STATE (as lbm_residual),
 * LBM_E_DEVICE. */
int lbm_check_into(lbm_ctx *ctx, double *out);

/* Copies the populations f_i(x, t) of the current time level (after
 * streaming, before collision) to / from host double[9][ny][nx].
 * set_populations replaces the state and synchronizes; get synchronizes.
 * Errors: LBM_E_DEVICE, LBM_E_NOMEM (staging buffer). */
int lbm_get_populations(lbm_ctx *ctx, double *f);
int lbm_set_populations(lbm_ctx *ctx, const double *f);

/* Obstacle mask: host unsigned char[ny][nx], nonzero = solid node; NULL
 * removes it.  A link whose source node is solid bounces back half-way with
 * the wall at rest (Sec. 5.2, Eq. 57-59 with u_w = 0); a link that leaves the
 * domain is handled by the face boundaries, never by the mask.  In the
 * density gradient a solid neighbour's density is replaced by the node's own,
 * as at a wall.  Solid nodes hold (and report) the rest state
 * feq(rho0, 0) and are left out of lbm_sums and lbm_residual.  The mask is
 * copied; it takes effect for every later call.  Synchronizes.
 * Errors: LBM_E_NOMEM, LBM_E_DEVICE. */
int lbm_set_mask(lbm_ctx *ctx, const unsigned char *mask);

/* Replaces the uniform body force (Eq. 13) for the following steps and for
 * the velocity definition rho u = sum f e + F/2 of later lbm_moments /
 * lbm_sums / lbm_residual calls.  Errors: LBM_E_INVAL (not finite). */
int lbm_set_force(lbm_ctx *ctx, double fx, double fy);

/* Enqueues n steps, step i driven by the force (fx[i], fy[i]) (host arrays;
 * fy may be NULL to keep the y component), as for a time-periodic force
 * F_m cos(w t) (Sec. 5.3).  The last force stays set.  Returns without
 * waiting.  Errors: LBM_E_INVAL (n < 0, fx NULL, a value not finite);
 * LBM_E_DEVICE. */
int lbm_step_forced(lbm_ctx *ctx, long n, const double *fx, const double *fy);

/* Advances one step and replaces the state by the mean of the states before
 * and after that step.  A mode that flips sign every step (the staggered
 * momentum of the D2Q9 streaming: x-momentum alternating from column to
 * column, y-momentum from row to row, which the momentum-conserving
 * collision cannot damp) cancels exactly; smooth fields move by half a step.
 * Meant for initial states set from macroscopic fields (lbm_set_fields
 * excites that mode whenever the fields are not the scheme's own steady
 * state).  Counts as one step; the residual needs a further step.
 * Synchronizes.  Errors: LBM_E_DEVICE, LBM_E_NOMEM. */
int lbm_smooth_step(lbm_ctx *ctx);

/* Replaces the relaxation rates omega_0..omega_8 (as in lbm_create) for the
 * following steps; the state is kept.  Synchronizes.
 * Errors: LBM_E_INVAL (a rate outside (0, 2)), LBM_E_DEVICE. */
int lbm_set_rates(lbm_ctx *ctx, const double rates[9]);

/* Streaming copy of `bytes` bytes from src to dst (device pointers, both
 * 16-byte aligned, bytes a multiple of 16) by the library's own kernel:
 * 16-byte loads and non-temporal 16-byte stores, grid-stride over
 * `workgroups` workgroups of 256 threads (0 = 8192).  It measures the
 * bandwidth that a plain read-plus-write stream reaches on this GPU, the
 * ceiling the step kernels are compared with.  Enqueues on `stream`
 * (hipStream_t, NULL = null stream) and returns without waiting.
 * Errors (text in lbm_last_error(NULL)): LBM_E_INVAL (NULL pointer,
 * misalignment, workgroups < 0), LBM_E_DEVICE. */
int lbm_stream_copy(void *dst, const void *src, size_t bytes, int workgroups, void *stream);

/* Number of steps taken since creation (set_fields / set_populations do not
 * reset it). */
long lbm_steps_done(const lbm_ctx *ctx);

/* Launch shape chosen for the step kernel: rows per wavefront and the number
 * of workgroups.  Errors: LBM_E_INVAL for a NULL ctx. */
int lbm_launch_shape(const lbm_ctx *ctx, int *rows_per_wave, int *workgroups);

/* Text of the last error of ctx (or of the last failed lbm_create when ctx is
 * NULL).  Never NULL; valid until the next call on the same context. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Releases the context and the buffers the library allocated (after
 * synchronizing its stream).  NULL is a no-op.  Returns LBM_OK. */
int lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
