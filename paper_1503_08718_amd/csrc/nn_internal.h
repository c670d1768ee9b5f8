// Internal interface of the warm-start network kernels (nn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrt {
struct ConvGeom {
    int n, D, H, W;
    int cin, cout, kpad;
    int circ;
};
hipError_t nn_conv_fwd(const void *in, const void *w, const float *bias, const ConvGeom &g, int relu, void *out,
                       float *out_f32, hipStream_t s);
hipError_t nn_weight_flip(const void *w, int cin, int cout, int kpad, int kpad_t, void *wt, hipStream_t s);
int nn_wgrad_splits(const ConvGeom &g);
int nn_wgrad_partials(const ConvGeom &g);
hipError_t nn_conv_wgrad(const void *x, const void *dy, const ConvGeom &g, int splits, float *partials, float *dw,
                         hipStream_t s);
hipError_t nn_bias_grad(const void *dy, long long nvox, int c, int splits, float *partials, float *db, hipStream_t s);
hipError_t nn_relu_bwd(const void *y, const void *dy, void *dx, long long n, hipStream_t s);
hipError_t nn_add(const void *a, const void *b, void *out, long long n, hipStream_t s);
hipError_t nn_pool2(int fwd, const void *in, int n, int D, int H, int W, int c, void *out, hipStream_t s);
hipError_t nn_up2(int fwd, const void *in, int n, int D, int H, int W, int c, void *out, hipStream_t s);
int nn_mse_blocks(long long nvox);
hipError_t nn_mse(const float *pred, int cpred, const float *target, long long nvox, void *dpred, float *partials,
                  hipStream_t s);
hipError_t nn_adam(float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
                   int t, void *wb, hipStream_t s);
hipError_t nn_to_bf16(const float *a, long long n, void *out, hipStream_t s);
hipError_t nn_features(const uint8_t *phase, int D, int H, int W, const float *feat, void *out, hipStream_t s);
hipError_t nn_features_resampled(const uint8_t *phase, int D, int H, int W, const float *feat, int Dc, int Hc, int Wc,
                                 void *out, hipStream_t s);
hipError_t nn_target(const float *T, int D, int H, int W, float scale, float *out, hipStream_t s);
int nn_temp_blocks(long long n);
hipError_t nn_to_temperature(const float *pred, int cpred, int Dc, int Hc, int Wc, int D, int H, int W, float scale,
                             float margin, float *T, int *bad, hipStream_t s);
// loss = scale * fixed-order sum of p[0 .. rows)
hipError_t nn_sum_rows(const float *p, int rows, float scale, float *out, hipStream_t s);
}  // namespace mrt
