// C ABI of the warm-start network layers (include/mrtlbm_nn.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/mrtlbm_nn.h"
#include "medium.h"
#include "nn_internal.h"



using namespace mrt;

static mrtlbm_status ret(hipError_t e, const char *what) { return e == hipSuccess ? MRTLBM_OK : hip_fail(e, what); }

static bool geom(int n, int d, int h, int w, int cin, int cout, int circ, ConvGeom *g) {
    if (n < 1 || d < 1 || h < 1 || w < 1 || cin < 8 || cin % 8 || cout < 16 || cout % 16 || circ < 0 || circ > 7)
        return false;
    if ((long long)n * d * h * w >= (1LL << 31)) return false;  // voxel indices are 32-bit in the kernels
    g->n = n; g->D = d; g->H = h; g->W = w;
    g->cin = cin; g->cout = cout;
    g->kpad = mrtlbm_nn_kpad(cin);
    g->circ = circ;
    return true;
}

extern "C" int mrtlbm_nn_kpad(int cin) { return (27 * cin + 31) / 32 * 32; }

extern "C" mrtlbm_status mrtlbm_nn_conv3d_fwd(const void *in, int n, int d, int h, int w, int cin, const void *weight,
                                              const float *bias, int cout, int circ, int relu, void *out,
                                              float *out_f32, void *stream) {
    ConvGeom g;
    if (!geom(n, d, h, w, cin, cout, circ, &g) || !in || !weight || (!out && !out_f32))
        return fail(MRTLBM_E_ARG, "conv3d_fwd: bad arguments");
    return ret(nn_conv_fwd(in, weight, bias, g, relu, out, out_f32, (hipStream_t)stream), "conv3d_fwd");
}

extern "C" mrtlbm_status mrtlbm_nn_conv3d_dgrad(const void *dout, int n, int d, int h, int w, int cin,
                                                const void *weight, int cout, int circ, void *wt_scratch, void *din,
                                                void *stream) {
    ConvGeom g;
    if (!geom(n, d, h, w, cin, cout, circ, &g) || !dout || !weight || !wt_scratch || !din || cin % 16)
        return fail(MRTLBM_E_ARG, "conv3d_dgrad: bad arguments (cin must be a multiple of 16)");
    hipStream_t s = (hipStream_t)stream;
    const int kpad_t = mrtlbm_nn_kpad(cout);
    hipError_t e = nn_weight_flip(weight, cin, cout, g.kpad, kpad_t, wt_scratch, s);
    if (e != hipSuccess) return hip_fail(e, "weight flip");
    // the adjoint is a convolution of dout with the flipped, transposed weights
    ConvGeom ga = g;
    ga.cin = cout;
    ga.cout = cin;
    ga.kpad = kpad_t;
    return ret(nn_conv_fwd(dout, wt_scratch, nullptr, ga, 0, din, nullptr, s), "conv3d_dgrad");
}

extern "C" size_t mrtlbm_nn_wgrad_scratch_bytes(int n, int d, int h, int w, int cin, int cout) {
    ConvGeom g;
    if (!geom(n, d, h, w, cin, cout, 0, &g)) return 0;
    const size_t a = (size_t)nn_wgrad_partials(g) * (size_t)cout * g.kpad * sizeof(float);
    const size_t b = (size_t)nn_wgrad_splits(g) * (size_t)cout * sizeof(float);
    return a > b ? a : b;
}

extern "C" mrtlbm_status mrtlbm_nn_conv3d_wgrad(const void *in, const void *dout, int n, int d, int h, int w, int cin,
                                                int cout, int circ, float *scratch, float *dw, float *db,
                                                void *stream) {
    ConvGeom g;
    if (!geom(n, d, h, w, cin, cout, circ, &g) || !in || !dout || !scratch || !dw)
        return fail(MRTLBM_E_ARG, "conv3d_wgrad: bad arguments");
    if (cout > 128) return fail(MRTLBM_E_ARG, "conv3d_wgrad: cout %d > 128", cout);
    hipStream_t s = (hipStream_t)stream;
    const int splits = nn_wgrad_splits(g);
    hipError_t e = nn_conv_wgrad(in, dout, g, splits, scratch, dw, s);
    if (e == hipSuccess && db) e = nn_bias_grad(dout, (long long)n * d * h * w, cout, splits, scratch, db, s);
    return ret(e, "conv3d_wgrad");
}

extern "C" mrtlbm_status mrtlbm_nn_relu_bwd(const void *y, const void *dy, void *dx, long long count, void *stream) {
    if (!y || !dy || !dx || count < 0) return fail(MRTLBM_E_ARG, "relu_bwd: bad arguments");
    return ret(nn_relu_bwd(y, dy, dx, count, (hipStream_t)stream), "relu_bwd");
}

extern "C" mrtlbm_status mrtlbm_nn_add(const void *a, const void *b, void *out, long long count, void *stream) {
    if (!a || !b || !out || count < 0) return fail(MRTLBM_E_ARG, "add: bad arguments");
    return ret(nn_add(a, b, out, count, (hipStream_t)stream), "add");
}

extern "C" mrtlbm_status mrtlbm_nn_pool2(int forward, const void *in, int n, int d, int h, int w, int c, void *out,
                                         void *stream) {
    if (!in || !out || n < 1 || d < 2 || h < 2 || w < 2 || (d | h | w) & 1 || c < 1)
        return fail(MRTLBM_E_ARG, "pool2: bad arguments");
    return ret(nn_pool2(forward, in, n, d, h, w, c, out, (hipStream_t)stream), "pool2");
}

extern "C" mrtlbm_status mrtlbm_nn_up2(int forward, const void *in, int n, int d, int h, int w, int c, void *out,
                                       void *stream) {
    if (!in || !out || n < 1 || d < 1 || h < 1 || w < 1 || c < 1) return fail(MRTLBM_E_ARG, "up2: bad arguments");
    return ret(nn_up2(forward, in, n, d, h, w, c, out, (hipStream_t)stream), "up2");
}

extern "C" mrtlbm_status mrtlbm_nn_mse(const float *pred, int cpred, const float *target, long long nvox, void *dpred,
                                       float *scratch, float *loss, void *stream) {
    if (!pred || !target || !dpred || !scratch || !loss || nvox < 1 || cpred < 1)
        return fail(MRTLBM_E_ARG, "mse: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = nn_mse(pred, cpred, target, nvox, dpred, scratch, s);
    // loss = fixed-order sum of the block partials / nvox
    if (e == hipSuccess) e = nn_sum_rows(scratch, nn_mse_blocks(nvox), 1.0f / (float)nvox, loss, s);
    return ret(e, "mse");
}

extern "C" mrtlbm_status mrtlbm_nn_adam(float *weight, const float *grad, float *m, float *v, long long count, float lr,
                                        float beta1, float beta2, float eps, int t, void *w_bf16, void *stream) {
    if (!weight || !grad || !m || !v || count < 0 || t < 1) return fail(MRTLBM_E_ARG, "adam: bad arguments");
    return ret(nn_adam(weight, grad, m, v, count, lr, beta1, beta2, eps, t, w_bf16, (hipStream_t)stream), "adam");
}

extern "C" mrtlbm_status mrtlbm_nn_to_bf16(const float *a, long long count, void *out, void *stream) {
    if (!a || !out || count < 0) return fail(MRTLBM_E_ARG, "to_bf16: bad arguments");
    return ret(nn_to_bf16(a, count, out, (hipStream_t)stream), "to_bf16");
}

extern "C" mrtlbm_status mrtlbm_nn_features(const unsigned char *phase, int d, int h, int w, const float *feat6,
                                            void *out, void *stream) {
    if (!phase || !feat6 || !out || d < 1 || h < 1 || w < 1) return fail(MRTLBM_E_ARG, "features: bad arguments");
    return ret(nn_features(phase, d, h, w, feat6, out, (hipStream_t)stream), "features");
}

extern "C" mrtlbm_status mrtlbm_nn_feature_table(const double *k6, int nphase, const double *spacing, float *out) {
    if (!k6 || !spacing || !out || nphase < 1 || nphase > 256) return fail(MRTLBM_E_ARG, "feature_table: bad arguments");
    for (int a = 0; a < 3; a++)
        if (!(spacing[a] > 0.0) || !std::isfinite(spacing[a])) return fail(MRTLBM_E_ARG, "feature_table: bad spacing");
    // change of variables x_a = spacing_a x'_a turns div(K grad T) = 0 into
    // the same equation in x' with K'_ab = K_ab / (spacing_a spacing_b)
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    std::vector<double> kt(6 * (size_t)nphase);
    double kmax = 0.0;
    for (int p = 0; p < nphase; p++) {
        double m[9], ev[3];
        for (int c = 0; c < 6; c++) kt[6 * p + c] = k6[6 * p + c] / (spacing[ia[c]] * spacing[ib[c]]);
        sym_full(&kt[6 * p], m);
        if (!sym_pd(m)) return fail(MRTLBM_E_TENSOR, "feature_table: tensor of phase %d is not positive definite", p);
        sym_eig(m, ev);
        kmax = std::max(kmax, std::max(ev[0], std::max(ev[1], ev[2])));
    }
    for (size_t i = 0; i < kt.size(); i++) out[i] = (float)(kt[i] / kmax);
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_nn_features_resampled(const unsigned char *phase, int d, int h, int w,
                                                      const float *feat6, int dc, int hc, int wc, void *out,
                                                      void *stream) {
    if (!phase || !feat6 || !out || d < 1 || h < 1 || w < 1 || dc < 1 || hc < 1 || wc < 1)
        return fail(MRTLBM_E_ARG, "features_resampled: bad arguments");
    return ret(nn_features_resampled(phase, d, h, w, feat6, dc, hc, wc, out, (hipStream_t)stream),
               "features_resampled");
}

extern "C" mrtlbm_status mrtlbm_nn_target(const float *t, int d, int h, int w, float scale, float *out, void *stream) {
    if (!t || !out || d < 1 || h < 1 || w < 1) return fail(MRTLBM_E_ARG, "target: bad arguments");
    return ret(nn_target(t, d, h, w, scale, out, (hipStream_t)stream), "target");
}

extern "C" mrtlbm_status mrtlbm_nn_to_temperature(const float *pred, int cpred, int dc, int hc, int wc, int d, int h,
                                                  int w, float scale, float margin, float *t, int *bad_scratch,
                                                  long long *bad_host, void *stream) {
    if (!pred || !t || !bad_scratch || !bad_host || cpred < 1 || dc < 1 || hc < 1 || wc < 1 || d < 1 || h < 1 ||
        w < 1 || scale == 0.0f)
        return fail(MRTLBM_E_ARG, "to_temperature: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const long long n = (long long)d * h * w;
    const int nb = nn_temp_blocks(n);
    hipError_t e = nn_to_temperature(pred, cpred, dc, hc, wc, d, h, w, scale, margin, t, bad_scratch, s);
    std::vector<int> counts(nb);
    if (e == hipSuccess) e = hipMemcpyAsync(counts.data(), bad_scratch, nb * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "to_temperature");
    long long bad = 0;
    for (int v : counts) bad += v;
    *bad_host = bad;
    return MRTLBM_OK;
}
