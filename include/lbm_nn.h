/*
 * lbm_nn.h -- C ABI of the kernels behind the learned warm start (same
 * library, liblbm.so): a convolutional encoder-decoder that maps an obstacle
 * mask and the flow parameters (Re, a) to a steady (rho, u, v) field, from
 * which the lattice of include/lbm.h starts (lbm_set_fields) instead of from
 * rest.  The lattice Boltzmann solver alone decides the result: the
 * network only chooses the initial state.
 *
 * Conventions
 *   - Tensors are NHWC, x fastest within a row, channels innermost.
 *   - Forward activations are BF16 (16-bit brain floats, passed as void *);
 *     gradients, biases, optimizer state and master weights are FP32.
 *   - A 3x3 convolution weight is FP32 W[k][co], k = tap * C + ci,
 *     tap = 3 (dy + 1) + (dx + 1): the output at (y, x) reads the input at
 *     (y + dy, x + dx) for dy, dx in {-1, 0, 1}, zero outside the image.
 *     The matrix cores read two BF16 copies made by lbm_nn_cast_weights:
 *     WT[co][k] (forward) and WD[ci][tap * cout + co] (data gradient).
 *   - A convolution may read the channel concatenation of two inputs
 *     (x1: c1 channels, then x2: c2 channels) without materializing it.
 *   - Every pointer is a device pointer unless stated; every call enqueues on
 *     `stream` (a hipStream_t, NULL = the null stream) and returns without
 *     waiting.  Returns LBM_NN_OK, LBM_NN_E_INVAL (checked before any work is
 *     enqueued) or LBM_NN_E_DEVICE (a launch failed).
 *   - 3x3 convolutions need c1, c2 (if present) and, for the gradients, cout
 *     to be multiples of 8, and 16-byte aligned tensors.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBM_NN_OK = 0, LBM_NN_E_INVAL = -1, LBM_NN_E_DEVICE = -3 };

/* y[n][h][w][cout] (BF16) = act(conv3x3(concat(x1, x2)) + bias); act = ReLU if
 * relu != 0, identity otherwise.  Implicit GEMM on the matrix cores (BF16
 * operands, FP32 accumulation). */
int lbm_nn_conv3x3_fwd(const void *x1, int c1, const void *x2, int c2, int n, int h, int w,
                       const void *wt, const float *bias, int cout, int relu, void *y,
                       void *stream);

/* Data gradient: gx1 / gx2 (FP32, c1 / c2 channels) = or += (accumulate != 0)
 * the gradient of the pre-activation output gy[n][h][w][cout] (FP32) through
 * the convolution with weights WD. */
int lbm_nn_conv3x3_dgrad(const float *gy, int n, int h, int w, int cout, const void *wd,
                         float *gx1, int c1, float *gx2, int c2, int accumulate, void *stream);

/* Weight and bias gradients: gw[9 (c1 + c2)][cout] and gb[cout] (FP32,
 * overwritten) of the pre-activation output gradient gy.  Deterministic
 * (fixed-order split reduction in `work`, at least
 * lbm_nn_conv3x3_wgrad_work(...) bytes). */
size_t lbm_nn_conv3x3_wgrad_work(int c1, int c2, int n, int h, int w, int cout);
int lbm_nn_conv3x3_wgrad(const void *x1, int c1, const void *x2, int c2, int n, int h, int w,
                         const float *gy, int cout, float *gw, float *gb, void *work,
                         size_t work_bytes, void *stream);

/* g[i] = gy[i] if y[i] > 0 else 0 (ReLU backward from the BF16 output y). */
int lbm_nn_relu_bwd(const float *gy, const void *y, float *g, size_t count, void *stream);

/* 2 x 2 average pooling of x[n][h][w][c] (BF16, h and w even) into
 * y[n][h/2][w/2][c]; backward spreads gy / 4 to gx[n][h][w][c] (= or +=). */
int lbm_nn_avgpool2_fwd(const void *x, int n, int h, int w, int c, void *y, void *stream);
int lbm_nn_avgpool2_bwd(const float *gy, int n, int h, int w, int c, float *gx, int accumulate,
                        void *stream);

/* Nearest upsampling by 2 of x[n][h][w][c] (BF16) into y[n][2h][2w][c];
 * backward sums the four copies: gx[n][h][w][c] = sum of gy over 2 x 2. */
int lbm_nn_upsample2_fwd(const void *x, int n, int h, int w, int c, void *y, void *stream);
int lbm_nn_upsample2_bwd(const float *gy, int n, int h, int w, int c, float *gx, void *stream);

/* 1x1 output head: y[m][cout] (FP32) = x[m][cin] (BF16) w[cin][cout] + b;
 * backward: gx[m][cin], gw[cin][cout], gb[cout] (FP32, overwritten), with a
 * fixed-order reduction in `work` (lbm_nn_conv1x1_work bytes). */
int lbm_nn_conv1x1_fwd(const void *x, int m, int cin, const float *w, const float *b, int cout,
                       float *y, void *stream);
size_t lbm_nn_conv1x1_work(int m, int cin, int cout);
int lbm_nn_conv1x1_bwd(const void *x, const float *gy, int m, int cin, const float *w, int cout,
                       float *gx, float *gw, float *gb, void *work, size_t work_bytes,
                       void *stream);

/* Masked mean-square error over m pixels x c channels:
 * loss = sum_{fluid pixels, channels} cw[ch] (pred - target)^2 / count, with
 * fluid[m] (uint8, 1 = counted); grad = d loss / d pred.  *loss is a device
 * float.  `work` holds lbm_nn_mse_work(m, c) bytes. */
size_t lbm_nn_mse_work(int m, int c);
int lbm_nn_mse(const float *pred, const float *target, const unsigned char *fluid, int m, int c,
               const float *cw, float count, float *grad, float *loss, void *work,
               size_t work_bytes, void *stream);

/* Adam (Kingma & Ba) on FP32 parameters p with moments m, v and gradient g,
 * bias-corrected for the 1-based step number. */
int lbm_nn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                float b2, float eps, int step, void *stream);

/* BF16 copies WT and WD of an FP32 3x3 weight W (c input, cout output channels). */
int lbm_nn_cast_weights(const float *w, int c, int cout, void *wt, void *wd, void *stream);

/* y[i] = BF16 of x[i]. */
int lbm_nn_cast_bf16(const float *x, size_t n, void *y, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NN_H */
