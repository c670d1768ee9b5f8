/*
 * mrtlbm_nn.h -- C ABI of the learned warm start: the layers of a small 3-D
 * convolutional encoder-decoder that maps a voxel medium to a starting
 * temperature field for the lattice Boltzmann solver of mrtlbm.h.  This is
 * not part of the paper's method: it only chooses the initial state, and the
 * solver itself always decides the converged result.
 *
 * Conventions:
 *   - Activations are BF16 (raw 16-bit patterns, `void *`), channels-last
 *     [n][d][h][w][c] with d = z, h = y, w = x.  Channel counts are multiples
 *     of 8 (inputs) and 16 (outputs of a convolution); a convolution takes
 *     n d h w < 2^31 voxels (E_ARG otherwise).
 *   - A 3x3x3 convolution's weights are BF16 [cout][kpad] with
 *     k = tap * cin + ci, tap = (dz * 3 + dy) * 3 + dx for offsets -1, 0, +1
 *     (cross-correlation), kpad = mrtlbm_nn_kpad(cin), entries k >= 27 cin
 *     zero.  Biases, master weights and gradients are FP32.
 *   - circ: bit 0 / 1 / 2 makes the x / y / z axis periodic; a clear bit pads
 *     that axis with zeros.
 *   - All pointers are device pointers owned by the caller, except those
 *     named *_host.  Work is enqueued on `stream` (a hipStream_t, NULL =
 *     default stream); calls that return host values synchronise it.
 *   - Products run on the matrix cores in BF16 with FP32 accumulation;
 *     reductions (weight and bias gradients, the loss) use fixed-order sums.
 *   - Status codes and mrtlbm_last_error() as in mrtlbm.h.
 */
#ifndef MRTLBM_NN_H
#define MRTLBM_NN_H

#include <stddef.h>

#include "mrtlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Padded length of a weight row: 32 * ceil(27 cin / 32). */
int mrtlbm_nn_kpad(int cin);

/* out[v][co] = act(bias[co] + sum_{tap, ci} w[co][tap cin + ci] in[v + off(tap)][ci]);
 * act = max(., 0) if relu.  Writes BF16 `out`, or FP32 `out_f32` if that is
 * not NULL.  bias may be NULL. */
mrtlbm_status mrtlbm_nn_conv3d_fwd(const void *in, int n, int d, int h, int w, int cin, const void *weight,
                                   const float *bias, int cout, int circ, int relu, void *out, float *out_f32,
                                   void *stream);

/* Gradient with respect to the input of mrtlbm_nn_conv3d_fwd (no activation):
 * din = adjoint convolution of dout.  wt_scratch: cin * mrtlbm_nn_kpad(cout)
 * BF16 values (the flipped, transposed weights). */
mrtlbm_status mrtlbm_nn_conv3d_dgrad(const void *dout, int n, int d, int h, int w, int cin, const void *weight,
                                     int cout, int circ, void *wt_scratch, void *din, void *stream);

/* FP32 scratch (bytes) needed by mrtlbm_nn_conv3d_wgrad. */
size_t mrtlbm_nn_wgrad_scratch_bytes(int n, int d, int h, int w, int cin, int cout);

/* Weight and bias gradients: dw[co][k] = sum_v dout[v][co] in[v + off(tap)][ci]
 * ([cout][kpad], padding entries 0), db[co] = sum_v dout[v][co]; db may be NULL.
 * cout <= 128 (E_ARG otherwise).  Voxel chunks are staged through LDS and
 * summed in a fixed order: the result does not depend on timing. */
mrtlbm_status mrtlbm_nn_conv3d_wgrad(const void *in, const void *dout, int n, int d, int h, int w, int cin, int cout,
                                     int circ, float *scratch, float *dw, float *db, void *stream);

/* dx = dy where y > 0, else 0 (backward of max(., 0) given its output y). */
mrtlbm_status mrtlbm_nn_relu_bwd(const void *y, const void *dy, void *dx, long long count, void *stream);

/* out = a + b (BF16, FP32 arithmetic). */
mrtlbm_status mrtlbm_nn_add(const void *a, const void *b, void *out, long long count, void *stream);

/* 2x2x2 average pooling (forward != 0) of in [n][d][h][w][c] into
 * [n][d/2][h/2][w/2][c], or its backward (in = gradient of the pooled grid,
 * out = gradient of the d x h x w grid).  d, h, w even. */
mrtlbm_status mrtlbm_nn_pool2(int forward, const void *in, int n, int d, int h, int w, int c, void *out, void *stream);

/* Nearest 2x upsampling (forward != 0) of in [n][d][h][w][c] into
 * [n][2d][2h][2w][c], or its backward (in = gradient of the fine grid). */
mrtlbm_status mrtlbm_nn_up2(int forward, const void *in, int n, int d, int h, int w, int c, void *out, void *stream);

/* Mean squared error of channel 0 of pred[v][cpred] (FP32) against
 * target[v]: loss[0] = mean (pred - target)^2; dpred (BF16 [v][cpred]) = its
 * gradient (zero on channels > 0).  scratch: 1024 floats. */
mrtlbm_status mrtlbm_nn_mse(const float *pred, int cpred, const float *target, long long nvox, void *dpred,
                            float *scratch, float *loss, void *stream);

/* One Adam step (moments m, v; bias correction with step t >= 1) on FP32
 * weights; w_bf16 (may be NULL) receives the updated weights in BF16. */
mrtlbm_status mrtlbm_nn_adam(float *weight, const float *grad, float *m, float *v, long long count, float lr,
                             float beta1, float beta2, float eps, int t, void *w_bf16, void *stream);

/* BF16 copy of FP32 values. */
mrtlbm_status mrtlbm_nn_to_bf16(const float *a, long long count, void *out, void *stream);

/* Network input for a medium with its gradient along x: out [d][h][w][8]
 * BF16 = (feat6[phase][0..5], (x + 1/2)/w - 1/2, 0), feat6 FP32 [nphase][6]. */
mrtlbm_status mrtlbm_nn_features(const unsigned char *phase, int d, int h, int w, const float *feat6, void *out,
                                 void *stream);

/* Host: per-phase network features of a medium sampled with voxel spacing
 * spacing[3] (x, y, z) relative to the network grid.  Each tensor k6[p]
 * (xx, yy, zz, xy, xz, yz) becomes K'_ab = K_ab / (spacing_a spacing_b) --
 * the conductivity that gives the same steady equation after the change of
 * variables x_a = spacing_a x'_a -- and all are divided by the largest
 * eigenvalue over the phases.  out: FP32 [nphase][6], host memory.
 * Errors: E_ARG, E_TENSOR (a transformed tensor not positive definite). */
mrtlbm_status mrtlbm_nn_feature_table(const double *k6, int nphase, const double *spacing, float *out);

/* Network input on a (dc, hc, wc) grid for a medium of (d, h, w) voxels with
 * its gradient along x: out [dc][hc][wc][8] BF16; channels 0..5 = mean of
 * feat6[phase] over the voxels whose centres lie in the coarse voxel (the
 * voxel under its centre when there are none), channel 6 = (x + 1/2)/wc - 1/2
 * of the coarse voxel, channel 7 = 0.  Equal sizes give mrtlbm_nn_features. */
mrtlbm_status mrtlbm_nn_features_resampled(const unsigned char *phase, int d, int h, int w, const float *feat6, int dc,
                                           int hc, int wc, void *out, void *stream);

/* Training target: out = scale * (T - T_lin(x)), T_lin = 1 - (x + 1/2)/w. */
mrtlbm_status mrtlbm_nn_target(const float *t, int d, int h, int w, float scale, float *out, void *stream);

/* Start field on the medium's (d, h, w) grid from a prediction made on a
 * (dc, hc, wc) grid spanning the same cell: trilinear interpolation of
 * channel 0 of pred [dc][hc][wc][cpred] between coarse voxel centres
 * (periodic in y and z, clamped in x), T = T_lin(x) + value / scale.
 * *bad_host = number of values that are not finite or lie outside
 * [-margin, 1 + margin] (the caller falls back to another start when it is
 * not 0).  bad_scratch: 2048 ints.  Synchronises. */
mrtlbm_status mrtlbm_nn_to_temperature(const float *pred, int cpred, int dc, int hc, int wc, int d, int h, int w,
                                       float scale, float margin, float *t, int *bad_scratch, long long *bad_host,
                                       void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MRTLBM_NN_H */
