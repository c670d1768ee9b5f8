// HBM copy ceiling: a plain streaming copy of `streams` separate arrays, the
// reference against which the step kernel's bandwidth is read.  The step
// kernel reads and writes 4 (moment storage) or 7 (population storage) state
// arrays per node; this kernel moves the same kind of 16-byte-per-lane
// streams with no arithmetic, so the ratio of the two isolates what the
// step's own work and access pattern cost.
#include <hip/hip_runtime.h>

#include "medium.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// every thread copies one 16-byte element of each of the S arrays: all S
// loads are issued before the first store
template <int S, bool NT>
__global__ void __launch_bounds__(256) k_stream_copy(const f4 *__restrict__ src, f4 *__restrict__ dst, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    f4 v[S];
#pragma unroll
    for (int k = 0; k < S; k++) v[k] = NT ? __builtin_nontemporal_load(src + k * n + i) : src[k * n + i];
#pragma unroll
    for (int k = 0; k < S; k++) {
        if constexpr (NT) __builtin_nontemporal_store(v[k], dst + k * n + i);
        else dst[k * n + i] = v[k];
    }
}

template <int S>
hipError_t launch(const f4 *src, f4 *dst, long long n, bool nt, hipStream_t s) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (nt) hipLaunchKernelGGL((k_stream_copy<S, true>), grid, dim3(256), 0, s, src, dst, n);
    else hipLaunchKernelGGL((k_stream_copy<S, false>), grid, dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace

extern "C" mrtlbm_status mrtlbm_stream_copy(const void *src_dev, void *dst_dev, long long n16, int streams, int nt,
                                            void *hip_stream) {
    if (!src_dev || !dst_dev) return mrt::fail(MRTLBM_E_ARG, "NULL argument");
    if (n16 < 1 || (n16 + 255) / 256 > 0x7fffffffLL) return mrt::fail(MRTLBM_E_ARG, "bad element count %lld", n16);
    if ((((uintptr_t)src_dev) | ((uintptr_t)dst_dev)) & 15) return mrt::fail(MRTLBM_E_ARG, "arrays not 16-byte aligned");
    const f4 *s = (const f4 *)src_dev;
    f4 *d = (f4 *)dst_dev;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    switch (streams) {
        case 1: e = launch<1>(s, d, n16, nt != 0, st); break;
        case 2: e = launch<2>(s, d, n16, nt != 0, st); break;
        case 4: e = launch<4>(s, d, n16, nt != 0, st); break;
        case 7: e = launch<7>(s, d, n16, nt != 0, st); break;
        default: return mrt::fail(MRTLBM_E_ARG, "streams must be 1, 2, 4 or 7 (got %d)", streams);
    }
    return e == hipSuccess ? MRTLBM_OK : mrt::hip_fail(e, "stream copy");
}
