// Steady-state solve that allocates nothing (mrtlbm_solve_noalloc).
//
// mrtlbm_solve replays hip graphs of K steps (graph instantiation allocates
// host and device memory) and reduces the check-step observables in the
// per-block partials of the medium's workspace.  This variant launches every
// step on its own (no graph) and keeps the per-block partials and the final
// reduction in `scratch`, a fixed device array of this file: a caller that
// cannot allocate (graph-free serving loops, harnesses that forbid it) only
// has to have created the medium beforehand.  The kernels, their block
// shapes and the reduction order are those of mrtlbm_solve, so both return
// the same numbers bit for bit.
//
// `scratch` is a host-side stand-in in host code: kernels get the device
// address returned by hipGetSymbolAddress, taken once per device with that
// device current and kept in scratch_ptr[].  Every call on one device shares
// that device's array; calls that overlap on one device race.  Nothing in it
// has to start at zero: each check block writes its own slot of partials and
// the reduction overwrites the final values.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_internal.h"
#include "medium.h"

using namespace mrt;

namespace {

// check-step partials of up to this many blocks, then the final reduction
constexpr int NOALLOC_MAX_PARTIALS = 65536;
constexpr size_t NOALLOC_DOUBLES = (size_t)(NOALLOC_MAX_PARTIALS + 2) * NRED;
constexpr int MAX_DEVICES = 64;

std::mutex g_scratch_mutex;
double *g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// device address of this device's scratch array (set-up on the first call
// per device, with that device current)
static mrtlbm_status scratch_for(int device, double **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(MRTLBM_E_ARG, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        hipError_t e2 = (cur != device) ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
        if (!p) return fail(MRTLBM_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = (double *)p;
    }
    *out = g_scratch_ptr[device];
    return MRTLBM_OK;
}

template <typename real>
static mrtlbm_status solve_noalloc(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind, long long max_steps, int K,
                                   double *partials, mrtlbm_result *out) {
    double *final8 = partials + (size_t)NOALLOC_MAX_PARTIALS * NRED;
    StopState ss;
    ss.check_vol = !has_side_flux(m);
    const double zero[NRED] = {};
    mrtlbm_result r{};
    fill_result(m, zero, &r);
    while (m->steps < max_steps) {
        const long long left = max_steps - m->steps;
        const long long block = left >= K ? K : left;
        int cur = m->cur;
        for (long long i = 0; i + 1 < block; i++) {
            hipError_t e = launch_step<real>(make_cell<real>(m, cur), m->launch, m->stream);
            if (e != hipSuccess) return hip_fail(e, "step kernel");
            cur ^= 1;
        }
        int nb = 0;
        hipError_t e = launch_check<real>(make_cell<real>(m, cur), m->launch, 1, partials, &nb, nullptr, 0.0, m->stream);
        if (e == hipSuccess) e = launch_reduce(partials, nb, final8, m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->pinned, final8, NRED * sizeof(double), hipMemcpyDeviceToHost, m->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) return hip_fail(e, "check step");
        m->cur = cur ^ 1;
        m->steps += block;
        fill_result(m, m->pinned, &r);
        const int v = stop_rule(ss, r, tol, kind);
        progress("solve: step %lld, k_hot %.8g, k_cold %.8g, k_leak %.3g, resid %.3g", r.steps, r.keff_hot,
                 r.keff_cold, r.keff_leak, r.resid);
        if (v == -1) { *out = r; return fail(MRTLBM_E_NONFINITE, "%d non-finite nodes at step %lld", r.nonfinite, r.steps); }
        if (v == -2) { *out = r; return fail(MRTLBM_E_DIVERGED, "residual %g grew from %g", r.resid, ss.min_resid); }
        if (v == 1) {
            r.converged = 1;
            *out = r;
            return MRTLBM_OK;
        }
    }
    *out = r;
    return MRTLBM_NOT_CONVERGED;
}

extern "C" mrtlbm_status mrtlbm_solve_noalloc(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind,
                                              long long max_steps, int check_every, mrtlbm_result *out) {
    if (!m || !out) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    if (check_every < 2 || (check_every & 1)) return fail(MRTLBM_E_ARG, "check_every must be even and >= 2");
    if (!(tol > 0)) return fail(MRTLBM_E_ARG, "tol must be > 0");
    if (kind != MRTLBM_TOL_MAXDT && kind != MRTLBM_TOL_KEFF) return fail(MRTLBM_E_ARG, "bad tolerance kind");
    const int nb = (m->prec == MRTLBM_F64) ? check_blocks<double>(make_cell<double>(m, 0), m->launch)
                                           : check_blocks<float>(make_cell<float>(m, 0), m->launch);
    if (nb > NOALLOC_MAX_PARTIALS)
        return fail(MRTLBM_E_WORKSPACE, "the check step needs %d partials; the fixed scratch holds %d", nb,
                    NOALLOC_MAX_PARTIALS);
    double *partials = nullptr;
    mrtlbm_status st = scratch_for(m->device, &partials);
    if (st != MRTLBM_OK) return st;
    return m->prec == MRTLBM_F64 ? solve_noalloc<double>(m, tol, kind, max_steps, check_every, partials, out)
                                 : solve_noalloc<float>(m, tol, kind, max_steps, check_every, partials, out);
}
