/*
 * mhdnn.h -- C ABI of the learned closure around the MHD path (gfx950).
 *
 * The closure corrects a coarse-grid run of the method: a small periodic 3D
 * convolutional network (3x3x3 kernels, channels 8 -> 32 -> 32 -> 8, GELU
 * between layers) maps the normalised coarse state to a correction that is
 * added after each coarse step.  It is trained on 4x box-filtered states of
 * fine-grid runs of the method itself.  The paper names machine-learned
 * reconstruction of turbulent flow only as related work (Section 6,
 * Discussion); the network, its training and its data recipe are this
 * library's own.
 *
 * Conventions
 *   - All array pointers are DEVICE pointers owned by the caller; `stream`
 *     is a hipStream_t (NULL = legacy default).  Calls are asynchronous.
 *   - Coarse grids are cubic with n in {16, 32, 64} cells per axis and
 *     periodic; a batch holds `batch` independent grids back to back.
 *   - Activations are channels-last BF16: element (b, cell, c) of a tensor
 *     with C channels is at (b*n^3 + cell)*C + c, cell = (k*n + j)*n + i.
 *   - Convolution weights for the kernels are BF16 laid out [32][27][cin]
 *     (output channels padded to 32 with zero rows); tap t covers offsets
 *     (dz, dy, dx) in {-1,0,1}^3 with t = 9(dz+1) + 3(dy+1) + (dx+1).
 *     FP32 master weights are [cout][27][cin].
 *   - Accumulation is FP32 on the MFMA units (v_mfma_f32_32x32x16_bf16).
 *   - Return values are MHD_OK (0) or MHD_ERR_INVALID (1) / MHD_ERR_DEVICE (3).
 */
#ifndef MHDNN_H
#define MHDNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 4x box filter: coarse[q][K][J][I] = mean of fine[q][4K+c][4J+b][4I+a],
 * a, b, c in 0..3, for the 8 fields of a fine state in the mhd_layout of
 * its context (`fine_ctx` from mhd_init; any precision).  `coarse` is FP32,
 * unpadded, field-major [8][n/4][n/4][n/4].  The fine grid must be cubic
 * with n divisible by 4.  Errors: MHD_ERR_INVALID. */
int mhdnn_box_filter4(const void *fine_ctx, const void *fine_fields, float *coarse,
                      void *stream);

/* Normalise and transpose 8 FP32 fields to channels-last BF16:
 * x[(b*n^3 + cell)*8 + q] = bf16((f[q][cell] - g[q][cell] - mean[q]) * inv_std[q]),
 * g = `sub` (same addressing as `src`; NULL: g = 0).  With `sub` the state
 * before a coarse step and `src` the state after it, the input is the
 * step's tendency.  The sources are addressed as src + b*batch_stride
 * + q*field_stride + origin + (k*plane + j)*row + i, so both an unpadded
 * field-major array (origin 0, row n, plane n*n) and a solver buffer (its
 * layout) work.  mean and inv_std are 8 host floats. */
int mhdnn_pack(const float *src, const float *sub, int64_t batch_stride, int64_t field_stride,
               int64_t origin, int64_t row, int64_t plane, int32_t n, int32_t batch,
               const float *mean, const float *inv_std, uint16_t *x_bf16, void *stream);

/* Periodic 3x3x3 convolution, implicit GEMM on MFMA.
 * y[cell][o] = bias[o] + sum_{t,c} w[o][t][c] x[cell + off(t)][c].
 * mode 0 (hidden layer): z_bf16 = y (pre-activation) and a_bf16 = GELU(y),
 *        both [cell][cout], GELU(x) = x (1 + erf(x / sqrt 2)) / 2;
 * mode 1 (output layer): y_f32 = y, [cell][cout].
 * cin in {8, 32}, cout in {8, 32}; unused outputs may be NULL. */
int mhdnn_conv3d_fwd(const uint16_t *x, const uint16_t *w_pad, const float *bias, int32_t n,
                     int32_t batch, int32_t cin, int32_t cout, int32_t mode, uint16_t *z_bf16,
                     uint16_t *a_bf16, float *y_f32, void *stream);

/* Data gradient through one convolution and the GELU below it:
 * dprev[cell][c] = GELU'(zprev[cell][c]) * sum_{t,o} w[o][t][c] dz[cell - off(t)][o],
 * evaluated as the same implicit GEMM with `wt_pad` = the transposed,
 * tap-flipped weights from mhdnn_prepare_weights.  cin_dz = channels of dz
 * (the layer's cout), cprev = the layer's cin. */
int mhdnn_conv3d_dgrad(const uint16_t *dz, const uint16_t *wt_pad, const uint16_t *zprev,
                       int32_t n, int32_t batch, int32_t cin_dz, int32_t cprev,
                       uint16_t *dprev, void *stream);

/* Weight and bias gradients of one convolution:
 * dw[o][t][c] = sum_cell dz[cell][o] x[cell + off(t)][c],  db[o] = sum_cell dz[cell][o],
 * FP32, deterministic (fixed-order split over cells).  `workspace` holds
 * mhdnn_wgrad_workspace_floats(n, batch) floats. */
int64_t mhdnn_wgrad_workspace_floats(int32_t n, int32_t batch);
int mhdnn_conv3d_wgrad(const uint16_t *x, const uint16_t *dz, int32_t n, int32_t batch,
                       int32_t cin, int32_t cout, float *workspace, float *dw, float *db,
                       void *stream);

/* mhdnn_conv3d_wgrad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bit for bit, with the per-block
 * partial sums in a library-owned device array of
 * MHDNN_WGRAD_SCRATCH_FLOATS floats (the partials of 512 blocks, 56.7 MB;
 * each GPU keeps its own copy until the process ends) instead of a caller
 * workspace.  Allocates nothing.  Sizes whose
 * mhdnn_wgrad_workspace_floats(n, batch) exceeds MHDNN_WGRAD_SCRATCH_FLOATS
 * are rejected with MHD_ERR_INVALID: every batch up to 32 at n = 64, up to
 * 128 at n = 32 and up to 512 at n = 16 fits, larger ones do not.  All
 * calls on one GPU share that array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must be serialised by the
 * caller.
 * Errors: MHD_ERR_INVALID (as mhdnn_conv3d_wgrad, and the size limit),
 * MHD_ERR_NO_DEVICE, MHD_ERR_DEVICE. */
#define MHDNN_WGRAD_SCRATCH_FLOATS (512LL * (27 * 32 * 32 + 32))
int mhdnn_conv3d_wgrad_noalloc(const uint16_t *x, const uint16_t *dz, int32_t n, int32_t batch,
                               int32_t cin, int32_t cout, float *dw, float *db, void *stream);

/* From FP32 master weights w[cout][27][cin], write the BF16 kernel layouts:
 * w_pad[32][27][cin] (zero rows for o >= cout) and, if wt_pad is not NULL,
 * wt_pad[32][27][cout] with wt_pad[c][t][o] = w[o][26 - t][c] (rows c >= cin zero). */
int mhdnn_prepare_weights(const float *w, int32_t cin, int32_t cout, uint16_t *w_pad,
                          uint16_t *wt_pad, void *stream);

/* Mean-squared error of one batch: y is the network output, channels-last
 * [b][cell][q] (batch * n^3 * 8 floats); the target is field-major
 * [b][q][cell] (the layout of mhdnn_pair's d) times tscale[q] (8 host
 * floats).  With e = y - target * tscale over all count = 8 batch n^3
 * elements: dy_bf16[b][cell][q] = bf16(2 e / count) and loss_partials[k]
 * (device, 256 floats) receives per-block partial sums of e^2 / count in a
 * fixed order (their sum is the loss).  n in {16, 32, 64}. */
int mhdnn_mse(const float *y, const float *target, const float *tscale, int32_t n,
              int32_t batch, uint16_t *dy_bf16, float *loss_partials, void *stream);

/* One training pair from a coarse step.  `stepped` is the coarse solver
 * state S after one step (the mhd_layout of `coarse_ctx`, FP32 storage)
 * taken from the filtered state c_now; c_now and c_next (the next filtered
 * state) are unpadded field-major [8][n^3].  Writes, field-major:
 * x_out = S - c_now (the step's tendency, the network input) and
 * d_out = c_next - S (what the coarse step misses, the target). */
int mhdnn_pair(const void *coarse_ctx, const void *stepped, const float *c_now,
               const float *c_next, float *x_out, float *d_out, void *stream);

/* Per-field mean and standard deviation (population, FP64, fixed order)
 * over npairs samples laid out [p][8][n3] (FP32):
 * mean_std[q] = mean of field q, mean_std[8 + q] = its standard deviation
 * (two passes).  `workspace` holds mhdnn_field_stats_workspace_doubles()
 * doubles; both are device memory. */
int64_t mhdnn_field_stats_workspace_doubles(void);
int mhdnn_field_stats(const float *x, int64_t npairs, int64_t n3, double *workspace,
                      double *mean_std, void *stream);

/* Adam (Kingma & Ba, bias-corrected) on n FP32 parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  t >= 1. */
int mhdnn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
               float b2, float eps, int32_t t, void *stream);

/* Add a network correction to the interior of a coarse solver state:
 * f[q][cell] += y[cell][q] * scale[q] (scale: 8 host floats), with the
 * compensated update of the FP32C variant when `comp` is not NULL.  `ctx`
 * is the coarse solver context (FP32 storage).
 * `guard` (device, 2 int32, may be NULL) makes the plain method the
 * fallback without a host round trip: the correction is applied only if
 * every corrected value (and compensation) of the call is finite, else the
 * state is left as the plain step left it and guard[1] is incremented
 * (the number of refused corrections; the caller zeroes it once).  guard[0]
 * is working space of the call.  Calls sharing a guard must not overlap. */
int mhdnn_apply(const void *ctx, void *fields, void *comp, const float *y, const float *scale,
                int32_t *guard, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MHDNN_H */
