/*
 * lbm_batch.h -- C ABI for batches of independent lattices advanced together
 * by the rectangular-lattice central moment LBM of include/lbm.h (same
 * library, liblbm.so).
 *
 * A batch holds many cases of uneven size, aspect ratio a = dy/dx, relaxation
 * rates, boundaries and forcing.  Each case is the scheme of include/lbm.h
 * (Sec. 3 / Sec. 4 collide-and-stream with the Sec. 5.2 boundaries), and its
 * results are bit-identical to a single lbm_ctx with the same parameters: the
 * batch only changes how the work is launched.  One step of the batch is one
 * launch of a persistent kernel that walks a device-resident list of
 * 64-column tiles of every active case; runs of steps are replayed from a
 * captured HIP graph.  Per-case residuals come from one batched,
 * deterministic FP64 reduction.
 *
 * Conventions are those of include/lbm.h (velocity ordering of Eq. 2, node
 * (i, j) at x = i, y = j a, host arrays double[ny][nx] / double[9][ny][nx],
 * int status returns, one thread per batch).
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One case: the arguments of lbm_create plus the per-case options. */
typedef struct {
    int nx, ny;          /* nodes, >= 3 each */
    double r;            /* aspect ratio a = dy/dx > 0 (Sec. 2.1) */
    double rates[9];     /* omega_0..omega_8 in (0, 2) (Eq. 5-6) */
    lbm_bc bc;           /* boundaries, as in lbm_create */
    double cs2;          /* 0 < cs2 < min(1, r^2); 0 selects min(1/3, 0.64 r^2) */
    double force[2];     /* uniform body force (Eq. 13) */
    double rho0;         /* reference density; 0 => 1 */
} lbm_case;

typedef struct {
    int collision;       /* LBM_RC (default) or LBM_RNR, for every case */
    int precision;       /* LBM_FP64 (default), LBM_FP32_DEV, LBM_FP64_DEV, LBM_FP32_DEV_F64 */
    int corrections;     /* 1 (default): Eq. 23-27 corrections on */
    int rows_per_wave;   /* rows marched by one wavefront, 1..64; 0 = automatic */
    int workgroups;      /* persistent grid size; 0 = automatic */
    int graph_steps;     /* steps per captured graph, even, >= 2; 0 => 64 */
    void *stream;        /* hipStream_t; NULL => the batch creates its own (graphs
                            cannot be captured on the null stream) */
    int tile_kernel;     /* 1: step with the one-node-per-thread tile kernel from the
                            start (the marching kernel while any case has a mask);
                            0 (default): the marching kernel until lbm_batch_autotune
                            chooses */
    int steps_per_launch; /* 0 (default, automatic) or 2: while no case has a mask,
                            advance pairs of steps with the two-steps-per-launch
                            kernel (lbm_set_steps_per_launch) on 64 x 8 block tiles,
                            the single steps with the tile kernel; 1: one step per
                            launch.  Results are bit-identical either way. */
    int two_step_form;   /* form of the two-step kernel (lbm_set_two_step_form):
                            LBM_FORM_AUTO (default: staged for LBM_FP32_DEV, else
                            register), LBM_FORM_REGISTER (64 x 8 block tiles) or
                            LBM_FORM_STAGED (64 x 24 block tiles, LBM_FP32_DEV only);
                            lbm_batch_autotune may change an automatic choice */
} lbm_batch_opts;

typedef struct lbm_batch lbm_batch;

void lbm_batch_default_opts(lbm_batch_opts *o);

/* Creates a batch of ncases >= 1 cases, every case at its rest equilibrium
 * f = feq(rho0, 0), all active.  The library allocates two buffers holding
 * every case (each case padded to 64-value rows, as lbm_required_bytes).
 * Errors: LBM_E_INVAL (a case fails the checks of lbm_create, with its index
 * in the message, or bad options); LBM_E_DEVICE; LBM_E_NOMEM.  *out is NULL
 * on error. */
int lbm_batch_create(int ncases, const lbm_case *cases, const lbm_batch_opts *opts,
                     lbm_batch **out);

/* f = feq(rho, u) for case c (as lbm_set_fields); the case's step count is
 * kept, its residual needs a step first.  Synchronizes.
 * Errors: LBM_E_INVAL (bad c), LBM_E_DEVICE. */
int lbm_batch_set_fields(lbm_batch *b, int c, const double *rho, const double *ux,
                         const double *uy);

/* Obstacle mask of case c (as lbm_set_mask): host unsigned char[ny][nx],
 * nonzero = solid; NULL removes it.  Synchronizes.
 * Errors: LBM_E_INVAL (bad c), LBM_E_NOMEM, LBM_E_DEVICE. */
int lbm_batch_set_mask(lbm_batch *b, int c, const unsigned char *mask);

/* lbm_smooth_step for every active case: one batched step, then each case's
 * state is replaced by the mean of its states before and after it.
 * Synchronizes.  Errors: LBM_E_DEVICE, LBM_E_NOMEM. */
int lbm_batch_smooth_step(lbm_batch *b);

/* Replaces the relaxation rates of case c for the following steps (as
 * lbm_set_rates).  A batch whose cases all had omega_6..8 = 1 at creation
 * runs the shorter collision for them, so they must stay 1.  Synchronizes.
 * Errors: LBM_E_INVAL, LBM_E_DEVICE. */
int lbm_batch_set_rates(lbm_batch *b, int c, const double rates[9]);

/* Marks which cases advance (active[c] != 0).  Inactive cases keep their state
 * and step count.  Takes effect for the next lbm_batch_step.
 * Errors: LBM_E_INVAL. */
int lbm_batch_set_active(lbm_batch *b, const int *active);

/* Advances every active case by n >= 0 steps (enqueued; does not wait).
 * Whole graph replays cover runs of graph_steps steps, single launches the
 * rest.  With two steps per launch (lbm_batch_steps_per_launch), pairs of
 * steps run while more than two steps remain and the call ends with one or
 * two single steps, so the residual of the last step is available.
 * Errors: LBM_E_INVAL (n < 0), LBM_E_DEVICE. */
int lbm_batch_step(lbm_batch *b, long n);

/* Per-case steady-state residual of the last step of each case,
 * R = sqrt(sum |u^n - u^(n-1)|^2) / sqrt(sum |u^n|^2) (FP64, deterministic),
 * into R[ncases].  Cases that have not stepped since their state was set get
 * -1; cases with NaN or Inf velocities get NaN (the call still returns LBM_OK).
 * Synchronizes.  Errors: LBM_E_DEVICE. */
int lbm_batch_residuals(lbm_batch *b, double *R);

/* Runs every active case until its residual, checked every check_every steps,
 * is <= tol, or it blows up, or max_steps steps have been taken by this call.
 * steps_out[ncases] (may be NULL) receives, per case, the number of steps this
 * call took to reach tol, -1 if the case blew up (it is then deactivated), or
 * -2 if it did not reach tol (or was inactive).  Converged cases are
 * deactivated.  Synchronizes.  Errors: LBM_E_INVAL, LBM_E_DEVICE. */
int lbm_batch_run_to_steady(lbm_batch *b, double tol, long check_every, long max_steps,
                            long *steps_out);

/* Case c's macroscopic fields / populations, as lbm_moments and
 * lbm_get_populations; set_populations as lbm_set_populations.
 * Synchronize.  Errors: LBM_E_INVAL (bad c), LBM_E_DEVICE, LBM_E_NOMEM. */
int lbm_batch_moments(lbm_batch *b, int c, double *rho, double *ux, double *uy);
int lbm_batch_get_populations(lbm_batch *b, int c, double *f);
int lbm_batch_set_populations(lbm_batch *b, int c, const double *f);

/* Steps taken by case c.  Returns -1 for a bad argument. */
long lbm_batch_steps_done(const lbm_batch *b, int c);

/* Times the batched step over candidate launch shapes (rows per wavefront x
 * persistent grid size of the marching kernel, and, when no case has a mask,
 * the one-node-per-thread tile kernel on 64 x 8 block tiles with three grid
 * sizes; it then reports 8 rows), trial_steps >= 1 launches each, and keeps
 * the fastest.  With two steps per launch in force it times only the
 * two-step kernel: its persistent grid (one block tile per workgroup, or a
 * few workgroups per CU) in each form allowed (the register form; the staged
 * form too for LBM_FP32_DEV unless two_step_form fixes one), and reports the
 * chosen form's block-tile rows (8 or 24).  Setting a mask later returns the batch to the marching
 * kernel.  The trial launches recompute one step from the current state
 * without committing it, so no case advances; the residual of every case
 * needs a step afterwards.  rows_out / workgroups_out (may be NULL) receive
 * the choice.  Synchronizes.  Errors: LBM_E_INVAL, LBM_E_DEVICE. */
int lbm_batch_autotune(lbm_batch *b, int trial_steps, int *rows_out, int *workgroups_out);

/* 1 if the batch steps with the tile kernel (chosen by lbm_batch_autotune
 * or taken with two steps per launch, when no case has a mask), 0 for the
 * marching kernel; -1 for a NULL batch. */
int lbm_batch_uses_tile_kernel(const lbm_batch *b);

/* Form of the batch's two-step kernel (LBM_FORM_REGISTER or LBM_FORM_STAGED);
 * LBM_E_INVAL for a NULL batch. */
int lbm_batch_two_step_form(const lbm_batch *b);

/* Steps per launch of the next long run: 2 while two steps per launch are
 * allowed (lbm_batch_opts.steps_per_launch) and no case has a mask, else 1;
 * LBM_E_INVAL for a NULL batch. */
int lbm_batch_steps_per_launch(const lbm_batch *b);

/* Current launch shape: rows per wavefront, persistent workgroups and the
 * number of tiles of the active cases.  Errors: LBM_E_INVAL. */
int lbm_batch_launch_shape(const lbm_batch *b, int *rows_per_wave, int *workgroups, int *tiles);

/* Text of the last error of b (or of the last failed lbm_batch_create when b
 * is NULL).  Never NULL. */
const char *lbm_batch_last_error(const lbm_batch *b);

/* Releases the batch (after synchronizing its stream).  NULL is a no-op. */
int lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_BATCH_H */
