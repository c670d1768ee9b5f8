// Host side of the C ABI declared in include/mrtlbm.h: per-medium setup
// (Eqs. 12-13), boundary description (Eqs. 23-25), the steady-state driver
// with FP64 observables (Eqs. 14-16, 22), checkpointing and the block-shape
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "lbm_internal.h"
#include "medium.h"

using namespace mrt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

mrtlbm_status mrt::fail(mrtlbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mrtlbm_status mrt::hip_fail(hipError_t e, const char *what) {
    return fail(MRTLBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *mrtlbm_last_error(void) { return g_err.c_str(); }

static mrtlbm_progress_fn g_progress = nullptr;
static void *g_progress_user = nullptr;
static double g_progress_interval = 30.0;
static std::chrono::steady_clock::time_point g_progress_last;

extern "C" void mrtlbm_set_progress(mrtlbm_progress_fn fn, void *user, double interval_s) {
    g_progress = fn;
    g_progress_user = user;
    g_progress_interval = interval_s > 0 ? interval_s : 0.0;
    g_progress_last = std::chrono::steady_clock::now();
}

void mrt::progress(const char *fmt, ...) {
    if (!g_progress) return;
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - g_progress_last).count() < g_progress_interval) return;
    g_progress_last = now;
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_progress(buf, g_progress_user);
}

#define HIPCHK(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// small symmetric 3x3 algebra (host, FP64)
// ---------------------------------------------------------------------------

// symmetric (xx, yy, zz, xy, xz, yz) -> row-major 3x3
void mrt::sym_full(const double *k6, double *m) {
    m[0] = k6[0]; m[4] = k6[1]; m[8] = k6[2];
    m[1] = m[3] = k6[3];
    m[2] = m[6] = k6[4];
    m[5] = m[7] = k6[5];
}

// eigenvalues of a symmetric 3x3 (trigonometric solution of the cubic)
void mrt::sym_eig(const double *m, double ev[3]) {
    const double p1 = m[1] * m[1] + m[2] * m[2] + m[5] * m[5];
    const double q = (m[0] + m[4] + m[8]) / 3.0;
    if (p1 == 0.0) {
        ev[0] = m[0]; ev[1] = m[4]; ev[2] = m[8];
        return;
    }
    const double p2 = (m[0] - q) * (m[0] - q) + (m[4] - q) * (m[4] - q) + (m[8] - q) * (m[8] - q) + 2.0 * p1;
    const double p = std::sqrt(p2 / 6.0);
    double b[9];
    for (int i = 0; i < 9; i++) b[i] = (m[i] - ((i % 4) == 0 ? q : 0.0)) / p;
    const double detb = b[0] * (b[4] * b[8] - b[5] * b[7]) - b[1] * (b[3] * b[8] - b[5] * b[6]) +
                        b[2] * (b[3] * b[7] - b[4] * b[6]);
    double r = detb / 2.0;
    r = std::min(1.0, std::max(-1.0, r));
    const double phi = std::acos(r) / 3.0;
    ev[0] = q + 2.0 * p * std::cos(phi);
    ev[2] = q + 2.0 * p * std::cos(phi + 2.0943951023931954923);
    ev[1] = 3.0 * q - ev[0] - ev[2];
}

// positive definite by Sylvester's criterion (leading minors)
bool mrt::sym_pd(const double *m) {
    const double d1 = m[0];
    const double d2 = m[0] * m[4] - m[1] * m[3];
    const double d3 = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                      m[2] * (m[3] * m[7] - m[4] * m[6]);
    return d1 > 0 && d2 > 0 && d3 > 0;
}

// inverse of a symmetric 3x3 by its adjugate
static void sym_inv(const double *m, double *inv) {
    const double c00 = m[4] * m[8] - m[5] * m[7];
    const double c01 = m[5] * m[6] - m[3] * m[8];
    const double c02 = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    inv[0] = c00 / det;
    inv[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    inv[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    inv[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    inv[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

// ---------------------------------------------------------------------------
// sizes and layout of the workspace
// ---------------------------------------------------------------------------

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t mrt::partial_capacity(int nx, int ny) { return (size_t)((nx + 15) / 16) * (size_t)ny + 4096; }

// the small arrays first, so that their offsets do not depend on the state
// storage; then the two state buffers of `values` reals per node
static bool layout(int nx, int ny, int nz, int nphase, mrtlbm_precision p, int values, size_t off[5],
                   size_t *total) {
    if (nx < 1 || ny < 1 || nz < 1 || nphase < 1 || nphase > 256) return false;
    if (nz > 65535 || (long long)ny > 65535LL * 16) return false;
    const size_t rs = (p == MRTLBM_F64) ? 8 : 4;
    const size_t N = (size_t)nx * ny * nz;
    size_t o = 0;
    off[2] = o; o = align256(o + partial_capacity(nx, ny) * NRED * 8); // partials
    off[3] = o; o = align256(o + 16 * 8);                              // final reduction
    off[4] = o; o = align256(o + (size_t)nphase * TABW * rs);          // phase tables
    off[0] = o; o = align256(o + values * N * rs);                     // buffer A
    off[1] = o; o = align256(o + values * N * rs);                     // buffer B
    *total = o;
    return true;
}

static int state_values_of(int storage) { return storage ? 4 : Q; }

extern "C" size_t mrtlbm_workspace_bytes_storage(int nx, int ny, int nz, int nphase, mrtlbm_precision p,
                                                 int storage) {
    size_t off[5], total;
    if ((p != MRTLBM_F32 && p != MRTLBM_F64) || (storage != 0 && storage != 1)) return 0;
    return layout(nx, ny, nz, nphase, p, state_values_of(storage), off, &total) ? total : 0;
}

extern "C" size_t mrtlbm_workspace_bytes(int nx, int ny, int nz, int nphase, mrtlbm_precision p) {
    return mrtlbm_workspace_bytes_storage(nx, ny, nz, nphase, p, 0);
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------

bool mrt::launch_ok(const mrtlbm_medium *m, const Launch &L) {
    if (L.vec != 1 && L.vec != 2 && L.vec != 4) return false;
    if (m->nx % L.vec) return false;
    if (L.bx != 8 && L.bx != 16 && L.bx != 32 && L.bx != 64) return false;
    const int t = L.bx * L.by;
    if (L.by < 1 || t < 64 || t > 256 || (t % 64)) return false;
    if (L.vec * L.bx < 16) return false;
    if (L.nt < 0 || L.nt > 3) return false;
    if (L.map < 0 || L.map > 1) return false;
    return true;
}

Launch mrt::default_launch(const mrtlbm_medium *m) {
    Launch L;
    if (m->prec == MRTLBM_F64) L.vec = (m->nx % 2 == 0) ? 2 : 1;
    else L.vec = (m->nx % 4 == 0) ? 4 : ((m->nx % 2 == 0) ? 2 : 1);
    const int nxv = m->nx / L.vec;
    int bx = 8;
    while (bx < 64 && bx < nxv) bx *= 2;
    while (L.vec * bx < 16) bx *= 2;
    L.bx = bx;
    L.by = 256 / bx;
    L.nt = 0;
    L.map = 0;
    return L;
}

// ---------------------------------------------------------------------------
// medium
// ---------------------------------------------------------------------------

template <typename real>
Cell<real> mrt::make_cell(const mrtlbm_medium *m, int cur) {
    Cell<real> c;
    c.src = (const real *)(cur ? m->bufB : m->bufA);
    c.dst = (real *)(cur ? m->bufA : m->bufB);
    c.phase = m->phase;
    c.tab = (const real *)m->tab;
    c.nx = m->nx; c.ny = m->ny; c.nz = m->nz;
    c.nxv = m->nx;
    c.N = m->N;
    c.nphase = m->nphase;
    const int ext[3] = {m->nx, m->ny, m->nz};
    const double dT = m->t_hot - m->t_cold;
    for (int a = 0; a < 3; a++) {
        const bool grad = (a == m->gaxis);
        c.per[a] = (!grad && m->side[a] == MRTLBM_PERIODIC) ? 1 : 0;
        c.sgn[a] = grad ? real(-1) : real(1);
        c.h[a] = grad ? (real)(0.25 * dT / (2.0 * ext[a])) : real(0);
    }
    c.gaxis = m->gaxis;
    c.storage = m->storage;
    c.relax = (m->tau_rest[0] != 1.0 || m->tau_rest[1] != 1.0 || m->tau_rest[2] != 1.0) ? 1 : 0;
    for (int i = 0; i < 3; i++) c.srel[i] = (real)(1.0 / m->tau_rest[i]);
    // Eq. 24 in lattice units: the inflow per link and step is s q
    for (int a = 0; a < 3; a++)
        for (int e = 0; e < 2; e++) c.phi[a][e] = (real)(m->s * m->qside[a][e]);
    return c;
}
template Cell<float> mrt::make_cell<float>(const mrtlbm_medium *, int);
template Cell<double> mrt::make_cell<double>(const mrtlbm_medium *, int);

static mrtlbm_status upload_tables(mrtlbm_medium *m) {
    // tau = I/2 + D / eps with D = s k and eps = 2 gamma = 1/4 (Eq. 13);
    // table row: half of (I - tau^-1), then tau - I
    double lmax = 0.0;
    for (int p = 0; p < m->nphase; p++) {
        double K[9], ev[3];
        sym_full(&m->k[6 * p], K);
        sym_eig(K, ev);
        lmax = std::max(lmax, std::max(ev[0], std::max(ev[1], ev[2])));
    }
    m->s = m->dmax * 0.25 / lmax;
    m->tab_host.assign((size_t)m->nphase * TABW, 0.0);
    for (int p = 0; p < m->nphase; p++) {
        double K[9], tau[9], A[9];
        sym_full(&m->k[6 * p], K);
        for (int i = 0; i < 9; i++) tau[i] = ((i % 4) == 0 ? 0.5 : 0.0) + m->s * K[i] / 0.25;
        sym_inv(tau, A);
        double *row = &m->tab_host[(size_t)p * TABW];
        const int ii[6] = {0, 4, 8, 1, 2, 5};
        for (int k = 0; k < 6; k++) {
            const double id = (k < 3) ? 1.0 : 0.0;
            row[k] = 0.5 * (id - A[ii[k]]);
            row[6 + k] = tau[ii[k]] - id;
        }
    }
    if (m->prec == MRTLBM_F64) {
        HIPCHK(hipMemcpyAsync(m->tab, m->tab_host.data(), m->tab_host.size() * 8, hipMemcpyHostToDevice, m->stream));
    } else {
        m->tab_host_f.resize(m->tab_host.size());
        for (size_t i = 0; i < m->tab_host.size(); i++) m->tab_host_f[i] = (float)m->tab_host[i];
        HIPCHK(hipMemcpyAsync(m->tab, m->tab_host_f.data(), m->tab_host_f.size() * 4, hipMemcpyHostToDevice,
                              m->stream));
    }
    HIPCHK(hipStreamSynchronize(m->stream));
    return MRTLBM_OK;
}

void mrt::drop_graphs(mrtlbm_medium *m) {
    for (auto &g : m->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    m->graphs.clear();
}

extern "C" mrtlbm_status mrtlbm_create(int nx, int ny, int nz, const unsigned char *phase_dev, const double *k_host,
                                       int nphase, mrtlbm_precision p, void *workspace_dev, size_t workspace_bytes,
                                       void *hip_stream, mrtlbm_medium **out) {
    if (!out) return fail(MRTLBM_E_ARG, "out is NULL");
    *out = nullptr;
    if (p != MRTLBM_F32 && p != MRTLBM_F64) return fail(MRTLBM_E_ARG, "bad precision %d", (int)p);
    size_t off[5], total, off7[5], total7;
    if (!layout(nx, ny, nz, nphase, p, 4, off, &total) || !layout(nx, ny, nz, nphase, p, Q, off7, &total7))
        return fail(MRTLBM_E_ARG, "bad sizes nx=%d ny=%d nz=%d nphase=%d", nx, ny, nz, nphase);
    if (!phase_dev || !k_host) return fail(MRTLBM_E_ARG, "phase_dev or k_host is NULL");
    if (!workspace_dev || workspace_bytes < total)
        return fail(MRTLBM_E_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, total);
    // a workspace that holds 7 populations per node starts in population
    // storage, a smaller one (moments only) in moment storage
    const int storage = workspace_bytes >= total7 ? 0 : 1;
    if (!storage) memcpy(off, off7, sizeof(off));
    if (((uintptr_t)workspace_dev) & 255) return fail(MRTLBM_E_WORKSPACE, "workspace not 256-byte aligned");
    for (int q = 0; q < nphase; q++) {
        double K[9];
        sym_full(k_host + 6 * q, K);
        bool finite = true;
        for (int i = 0; i < 6; i++) finite = finite && std::isfinite(k_host[6 * q + i]);
        if (!finite || !sym_pd(K)) return fail(MRTLBM_E_TENSOR, "tensor of phase %d is not positive definite", q);
    }
    auto *m = new mrtlbm_medium();
    m->nx = nx; m->ny = ny; m->nz = nz;
    m->N = (long long)nx * ny * nz;
    m->nphase = nphase;
    m->prec = p;
    m->phase = phase_dev;
    m->k.assign(k_host, k_host + 6 * nphase);
    m->dmax = 1.0;
    m->gaxis = 0; m->t_hot = 1.0; m->t_cold = 0.0;
    m->side[0] = m->side[1] = m->side[2] = MRTLBM_PERIODIC;
    m->ws = workspace_dev;
    m->ws_bytes = workspace_bytes;
    char *w = (char *)workspace_dev;
    m->bufA = w + off[0];
    m->bufB = w + off[1];
    m->partials = (double *)(w + off[2]);
    m->final8 = (double *)(w + off[3]);
    m->tab = w + off[4];
    m->storage = storage;
    m->pcap = partial_capacity(nx, ny);
    m->stream = (hipStream_t)hip_stream;
    m->launch = default_launch(m);
    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&m->pinned, 256, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "hipHostMalloc");
    }
    // phase ids < nphase, checked on the device
    const int nb = (int)std::min<long long>(1024, std::max<long long>(1, (m->N + 255) / 256));
    int *bm = (int *)m->partials;
    e = launch_phase_max(phase_dev, m->N, bm, nb, m->stream);
    std::vector<int> hbm(nb);
    if (e == hipSuccess) e = hipMemcpyAsync(hbm.data(), bm, nb * sizeof(int), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        mrtlbm_destroy(m);
        return hip_fail(e, "phase scan");
    }
    const int mx = *std::max_element(hbm.begin(), hbm.end());
    if (mx >= nphase) {
        mrtlbm_destroy(m);
        return fail(MRTLBM_E_ARG, "phase id %d >= nphase %d", mx, nphase);
    }
    mrtlbm_status st = upload_tables(m);
    if (st != MRTLBM_OK) {
        mrtlbm_destroy(m);
        return st;
    }
    *out = m;
    return MRTLBM_OK;
}

extern "C" void mrtlbm_destroy(mrtlbm_medium *m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    else (void)hipDeviceSynchronize();
    drop_graphs(m);
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    if (m->ev0) (void)hipEventDestroy(m->ev0);
    if (m->ev1) (void)hipEventDestroy(m->ev1);
    if (m->pinned) (void)hipHostFree(m->pinned);
    delete m;
}

extern "C" mrtlbm_status mrtlbm_set_bc(mrtlbm_medium *m, int grad_axis, double t_hot, double t_cold,
                                       const int side[3]) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (grad_axis < 0 || grad_axis > 2) return fail(MRTLBM_E_BC, "grad_axis %d", grad_axis);
    if (!std::isfinite(t_hot) || !std::isfinite(t_cold) || t_hot == t_cold)
        return fail(MRTLBM_E_BC, "wall temperatures must be finite and differ");
    if (!side) return fail(MRTLBM_E_BC, "side is NULL");
    for (int a = 0; a < 3; a++)
        if (a != grad_axis && side[a] != MRTLBM_PERIODIC && side[a] != MRTLBM_ADIABATIC)
            return fail(MRTLBM_E_BC, "side[%d] = %d", a, side[a]);
    m->gaxis = grad_axis;
    m->t_hot = t_hot;
    m->t_cold = t_cold;
    for (int a = 0; a < 3; a++) m->side[a] = (a == grad_axis) ? MRTLBM_PERIODIC : side[a];
    for (int a = 0; a < 3; a++) m->qside[a][0] = m->qside[a][1] = 0.0;
    m->initialised = false;
    drop_graphs(m);
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_set_side_flux(mrtlbm_medium *m, int axis, double q_lo, double q_hi) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (axis < 0 || axis > 2 || axis == m->gaxis) return fail(MRTLBM_E_BC, "side flux on axis %d", axis);
    if (m->side[axis] != MRTLBM_ADIABATIC) return fail(MRTLBM_E_BC, "axis %d has no Neumann faces", axis);
    if (!std::isfinite(q_lo) || !std::isfinite(q_hi)) return fail(MRTLBM_E_ARG, "side flux not finite");
    m->qside[axis][0] = q_lo;
    m->qside[axis][1] = q_hi;
    drop_graphs(m);
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_set_relaxation(mrtlbm_medium *m, double tau4, double tau5, double tau6) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    const double t[3] = {tau4, tau5, tau6};
    for (int i = 0; i < 3; i++)
        if (!(t[i] > 0.5) || !std::isfinite(t[i])) return fail(MRTLBM_E_ARG, "tau_%d = %g must exceed 1/2", i + 4, t[i]);
    if (m->storage && (tau4 != 1.0 || tau5 != 1.0 || tau6 != 1.0))
        return fail(MRTLBM_E_ARG, "moment storage holds only tau_4 = tau_5 = tau_6 = 1");
    for (int i = 0; i < 3; i++) m->tau_rest[i] = t[i];
    drop_graphs(m);
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_set_scale(mrtlbm_medium *m, double dmax) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (!(dmax > 0.0 && dmax <= 1.5)) return fail(MRTLBM_E_ARG, "dmax %g outside (0, 1.5]", dmax);
    m->dmax = dmax;
    m->initialised = false;
    drop_graphs(m);
    return upload_tables(m);
}

extern "C" mrtlbm_status mrtlbm_info(const mrtlbm_medium *m, double *scale, long long *steps, mrtlbm_launch *launch) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (scale) *scale = m->s;
    if (steps) *steps = m->steps;
    if (launch) {
        launch->vec = m->launch.vec; launch->bx = m->launch.bx; launch->by = m->launch.by; launch->nt = m->launch.nt;
        launch->map = m->launch.map;
    }
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_set_launch(mrtlbm_medium *m, const mrtlbm_launch *launch) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    Launch L = launch ? Launch{launch->vec, launch->bx, launch->by, launch->nt, launch->map} : default_launch(m);
    if (!launch_ok(m, L))
        return fail(MRTLBM_E_ARG, "launch shape vec=%d bx=%d by=%d nt=%d not admissible", L.vec, L.bx, L.by, L.nt);
    drop_graphs(m);
    m->launch = L;
    return MRTLBM_OK;
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------

template <typename real>
static hipError_t plain_steps(mrtlbm_medium *m, long long n, hipStream_t s, int *cur) {
    for (long long i = 0; i < n; i++) {
        hipError_t e = launch_step<real>(make_cell<real>(m, *cur), m->launch, s);
        if (e != hipSuccess) return e;
        *cur ^= 1;
    }
    return hipSuccess;
}

template <typename real>
static hipError_t check_step(mrtlbm_medium *m, int mode, hipStream_t s, int *cur, void *qout, double qscale) {
    const Cell<real> c = make_cell<real>(m, *cur);
    if ((size_t)check_blocks<real>(c, m->launch) > m->pcap) return hipErrorInvalidValue;
    int nb = 0;
    hipError_t e = launch_check<real>(c, m->launch, mode, m->partials, &nb, (real *)qout, qscale, s);
    if (e != hipSuccess) return e;
    e = launch_reduce(m->partials, nb, m->final8, s);
    if (e != hipSuccess) return e;
    if (mode == 1) *cur ^= 1;
    return hipSuccess;
}

// Graph of `K` steps starting from buffer parity `cur`: K-1 plain steps, then
// (if with_check) one step that also evaluates the observables, the final
// reduction and a copy of the 8 doubles to pinned host memory.
template <typename real>
static mrtlbm_status get_graph(mrtlbm_medium *m, int K, bool with_check, hipGraphExec_t *exec) {
    for (auto &g : m->graphs)
        if (g.K == K && g.cur == m->cur && g.check == with_check) {
            *exec = g.exec;
            return MRTLBM_OK;
        }
    if (!m->cap_stream) HIPCHK(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    int cur = m->cur;
    hipError_t e = plain_steps<real>(m, with_check ? K - 1 : K, m->cap_stream, &cur);
    if (e == hipSuccess && with_check) e = check_step<real>(m, 1, m->cap_stream, &cur, nullptr, 0.0);
    if (e == hipSuccess && with_check)
        e = hipMemcpyAsync(m->pinned, m->final8, NRED * sizeof(double), hipMemcpyDeviceToHost, m->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(m->cap_stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(e, "graph capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    if (m->graphs.size() >= 8) drop_graphs(m);
    m->graphs.push_back(GraphEntry{K, m->cur, with_check, graph, ge});
    *exec = ge;
    return MRTLBM_OK;
}

template <typename real>
static mrtlbm_status do_steps(mrtlbm_medium *m, long long nsteps) {
    const int G = 64;
    long long done = 0;
    if (nsteps >= 2 * G) {
        hipGraphExec_t ge;
        mrtlbm_status st = get_graph<real>(m, G, false, &ge);
        if (st != MRTLBM_OK) return st;
        for (; done + G <= nsteps; done += G) HIPCHK(hipGraphLaunch(ge, m->stream));
    }
    int cur = m->cur;
    HIPCHK(plain_steps<real>(m, nsteps - done, m->stream, &cur));
    m->cur = cur;
    m->steps += nsteps;
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_step(mrtlbm_medium *m, long long nsteps) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised (call mrtlbm_init)");
    if (nsteps < 0) return fail(MRTLBM_E_ARG, "nsteps < 0");
    return m->prec == MRTLBM_F64 ? do_steps<double>(m, nsteps) : do_steps<float>(m, nsteps);
}

extern "C" mrtlbm_status mrtlbm_init(mrtlbm_medium *m, const void *t0_dev, int flags) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    const double dT = m->t_hot - m->t_cold;
    hipError_t e;
    if (m->prec == MRTLBM_F64)
        e = launch_init<double>(make_cell<double>(m, 0), (double *)m->bufA, (const double *)t0_dev, flags, m->t_hot, dT,
                                m->stream);
    else
        e = launch_init<float>(make_cell<float>(m, 0), (float *)m->bufA, (const float *)t0_dev, flags, m->t_hot, dT,
                               m->stream);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    m->cur = 0;
    m->steps = 0;
    m->initialised = true;
    return MRTLBM_OK;
}

// ---------------------------------------------------------------------------
// observables
// ---------------------------------------------------------------------------

void mrt::fill_result(const mrtlbm_medium *m, const double *f, mrtlbm_result *out) {
    const int ext[3] = {m->nx, m->ny, m->nz};
    const double ng = ext[m->gaxis];
    const double area = (double)m->N / ng;
    const double dT = m->t_hot - m->t_cold;
    const double s = m->s;
    out->keff_hot = ng * f[R_PHI_HOT] / (dT * area * s);
    out->keff_cold = ng * f[R_PHI_COLD] / (dT * area * s);
    for (int a = 0; a < 3; a++) out->keff_col[a] = ng * (f[R_QX + a] / (double)m->N) / (dT * s);
    out->keff_vol = out->keff_col[m->gaxis];
    out->keff = 0.5 * (out->keff_hot + out->keff_cold);
    out->resid = f[R_RESID];
    out->temp_mean = f[R_TSUM] / (double)m->N + 0.5 * (m->t_hot + m->t_cold);
    out->nonfinite = (int)f[R_NONFINITE];
    out->keff_leak = ng * f[R_LEAK] / (dT * area * s);
    // heat imposed through Neumann faces, in the same units: s q per link,
    // one link per node of the face
    double side_in = 0.0;
    for (int a = 0; a < 3; a++) side_in += (m->qside[a][0] + m->qside[a][1]) * ((double)m->N / ext[a]);
    out->keff_side = ng * side_in / (dT * area);
    out->steps = m->steps;
    out->converged = 0;
}

extern "C" mrtlbm_status mrtlbm_keff(mrtlbm_medium *m, mrtlbm_result *out) {
    if (!m || !out) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    int cur = m->cur;
    hipError_t e = (m->prec == MRTLBM_F64) ? check_step<double>(m, 2, m->stream, &cur, nullptr, 0.0)
                                           : check_step<float>(m, 2, m->stream, &cur, nullptr, 0.0);
    if (e != hipSuccess) return hip_fail(e, "observables");
    HIPCHK(hipMemcpyAsync(m->pinned, m->final8, NRED * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    fill_result(m, m->pinned, out);
    return out->nonfinite ? fail(MRTLBM_E_NONFINITE, "%d non-finite nodes", out->nonfinite) : MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_flux(mrtlbm_medium *m, void *q_dev) {
    if (!m || !q_dev) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    int cur = m->cur;
    hipError_t e = (m->prec == MRTLBM_F64) ? check_step<double>(m, 3, m->stream, &cur, q_dev, 1.0 / m->s)
                                           : check_step<float>(m, 3, m->stream, &cur, q_dev, 1.0 / m->s);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "flux field");
}

extern "C" mrtlbm_status mrtlbm_temperature(mrtlbm_medium *m, void *t_dev) {
    if (!m || !t_dev) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    const double dT = m->t_hot - m->t_cold;
    hipError_t e;
    if (m->prec == MRTLBM_F64)
        e = launch_temperature<double>(make_cell<double>(m, m->cur), (const double *)(m->cur ? m->bufB : m->bufA),
                                       (double *)t_dev, m->t_hot, dT, m->stream);
    else
        e = launch_temperature<float>(make_cell<float>(m, m->cur), (const float *)(m->cur ? m->bufB : m->bufA),
                                      (float *)t_dev, m->t_hot, dT, m->stream);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "temperature kernel");
}

// stop rule shared by the single and the batched driver
bool mrt::has_side_flux(const mrtlbm_medium *m) {
    for (int a = 0; a < 3; a++)
        if (m->qside[a][0] != 0.0 || m->qside[a][1] != 0.0) return true;
    return false;
}

int mrt::stop_rule(StopState &ss, const mrtlbm_result &r, double tol, mrtlbm_tol_kind kind) {
    if (r.nonfinite) return -1;
    if (ss.min_resid > 0 && r.resid > 1e3 * ss.min_resid && r.resid > 1e-6) return -2;
    if (ss.min_resid < 0 || r.resid < ss.min_resid) ss.min_resid = r.resid;
    if (kind == MRTLBM_TOL_MAXDT) return r.resid < tol ? 1 : 0;
    // energy accumulation rate through the walls and the Neumann faces plus
    // the exact rounding energy of the stored state: dE/dt of the stored
    // field, relative to the through-flux (equal to the plain wall-flux gap
    // in exact arithmetic without side inflow)
    const double km = r.keff, ak = std::fabs(km);
    const bool gap_ok = std::fabs(r.keff_hot - r.keff_cold + r.keff_side + r.keff_leak) < tol * ak;
    // the volume mean of the node flux averages every plane's flux; at steady
    // state it equals the wall mean.  A transient mode that leaves the stored
    // energy unchanged (it moves heat from one part of the cell to another)
    // has equal wall fluxes, so the balance above misses it, but its plane
    // fluxes differ inside the cell and pull the volume mean away (with heat
    // imposed through side faces the plane fluxes differ at steady state too,
    // and this test is off)
    const bool vol_ok = !ss.check_vol || std::fabs(r.keff_vol - km) < tol * ak;
    // remaining change of k: the last change d between checks, extended by
    // its geometric tail d r / (1 - r), r = |d| / |previous d| (the slowest
    // mode decays geometrically); from a zero start T rises monotonically and
    // the gap alone bounds the error, from any other start this tail does
    bool chg_ok = false;
    if (ss.have_prev) {
        const double d = km - ss.kprev;
        if (std::fabs(d) < 1e-3 * tol * ak) {
            chg_ok = true;  // change at round-off level
        } else if (ss.have_d) {
            const double ratio = std::fabs(d) / std::max(std::fabs(ss.dprev), 1e-300);
            const double tail = ratio < 0.999 ? std::fabs(d) * ratio / (1.0 - ratio) : 1e300;
            chg_ok = std::max(std::fabs(d), tail) < 0.25 * tol * ak;
        }
        ss.dprev = d;
        ss.have_d = true;
    }
    ss.kprev = km;
    ss.have_prev = true;
    // two checks in a row, so that a turning point of k(t) that happens to
    // meet the balance does not end the run
    ss.passes = (gap_ok && vol_ok && chg_ok) ? ss.passes + 1 : 0;
    return ss.passes >= 2 ? 1 : 0;
}

template <typename real>
static mrtlbm_status do_solve(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind, long long max_steps, int K,
                              mrtlbm_result *out) {
    StopState ss;
    ss.check_vol = !has_side_flux(m);
    mrtlbm_result r{};
    fill_result(m, std::vector<double>(NRED, 0.0).data(), &r);
    while (m->steps < max_steps) {
        const long long left = max_steps - m->steps;
        if (left >= K) {
            hipGraphExec_t ge;
            mrtlbm_status st = get_graph<real>(m, K, true, &ge);
            if (st != MRTLBM_OK) return st;
            HIPCHK(hipGraphLaunch(ge, m->stream));
            m->steps += K;
        } else {
            int cur = m->cur;
            HIPCHK(plain_steps<real>(m, left - 1, m->stream, &cur));
            HIPCHK(check_step<real>(m, 1, m->stream, &cur, nullptr, 0.0));
            HIPCHK(hipMemcpyAsync(m->pinned, m->final8, NRED * sizeof(double), hipMemcpyDeviceToHost, m->stream));
            m->cur = cur;
            m->steps += left;
        }
        HIPCHK(hipStreamSynchronize(m->stream));
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

extern "C" mrtlbm_status mrtlbm_solve(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind, long long max_steps,
                                      int check_every, mrtlbm_result *out) {
    if (!m || !out) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    if (check_every < 2 || (check_every & 1)) return fail(MRTLBM_E_ARG, "check_every must be even and >= 2");
    if (!(tol > 0)) return fail(MRTLBM_E_ARG, "tol must be > 0");
    if (kind != MRTLBM_TOL_MAXDT && kind != MRTLBM_TOL_KEFF) return fail(MRTLBM_E_ARG, "bad tolerance kind");
    return m->prec == MRTLBM_F64 ? do_solve<double>(m, tol, kind, max_steps, check_every, out)
                                 : do_solve<float>(m, tol, kind, max_steps, check_every, out);
}

// ---------------------------------------------------------------------------
// checkpoint / resume
// ---------------------------------------------------------------------------

extern "C" int mrtlbm_state_values(const mrtlbm_medium *m) { return !m ? 0 : (m->storage ? 4 : Q); }

extern "C" mrtlbm_status mrtlbm_set_storage(mrtlbm_medium *m, int storage) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    if (storage != 0 && storage != 1) return fail(MRTLBM_E_ARG, "storage must be 0 or 1");
    if (storage == 1 && (m->tau_rest[0] != 1.0 || m->tau_rest[1] != 1.0 || m->tau_rest[2] != 1.0))
        return fail(MRTLBM_E_ARG, "moment storage holds only tau_4 = tau_5 = tau_6 = 1");
    size_t off[5], total;
    layout(m->nx, m->ny, m->nz, m->nphase, m->prec, state_values_of(storage), off, &total);
    if (total > m->ws_bytes)
        return fail(MRTLBM_E_WORKSPACE, "workspace of %zu bytes, storage %d needs %zu", m->ws_bytes, storage, total);
    m->bufA = (char *)m->ws + off[0];
    m->bufB = (char *)m->ws + off[1];
    m->storage = storage;
    m->initialised = false;
    drop_graphs(m);
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_state_get(mrtlbm_medium *m, void *f_dev) {
    if (!m || !f_dev) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    const size_t bytes = (size_t)mrtlbm_state_values(m) * m->N * (m->prec == MRTLBM_F64 ? 8 : 4);
    HIPCHK(hipMemcpyAsync(f_dev, m->cur ? m->bufB : m->bufA, bytes, hipMemcpyDeviceToDevice, m->stream));
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_state_set(mrtlbm_medium *m, const void *f_dev, long long steps) {
    if (!m || !f_dev) return fail(MRTLBM_E_ARG, "NULL argument");
    if (steps < 0) return fail(MRTLBM_E_ARG, "steps < 0");
    const size_t bytes = (size_t)mrtlbm_state_values(m) * m->N * (m->prec == MRTLBM_F64 ? 8 : 4);
    HIPCHK(hipMemcpyAsync(m->bufA, f_dev, bytes, hipMemcpyDeviceToDevice, m->stream));
    m->cur = 0;
    m->steps = steps;
    m->initialised = true;
    return MRTLBM_OK;
}

// ---------------------------------------------------------------------------
// timing and autotuning
// ---------------------------------------------------------------------------

extern "C" mrtlbm_status mrtlbm_time_steps(mrtlbm_medium *m, long long nsteps, double *ms) {
    if (!m || !ms) return fail(MRTLBM_E_ARG, "NULL argument");
    if (!m->initialised) return fail(MRTLBM_E_ARG, "state not initialised");
    if (!m->ev0) HIPCHK(hipEventCreate(&m->ev0));
    if (!m->ev1) HIPCHK(hipEventCreate(&m->ev1));
    HIPCHK(hipEventRecord(m->ev0, m->stream));
    mrtlbm_status st = mrtlbm_step(m, nsteps);
    if (st != MRTLBM_OK) return st;
    HIPCHK(hipEventRecord(m->ev1, m->stream));
    HIPCHK(hipEventSynchronize(m->ev1));
    float f = 0;
    HIPCHK(hipEventElapsedTime(&f, m->ev0, m->ev1));
    *ms = f;
    return MRTLBM_OK;
}

static std::string tune_key(const mrtlbm_medium *m) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, m->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    std::ostringstream k;
    k << arch << ' ' << m->nx << ' ' << m->ny << ' ' << m->nz << ' ' << (m->prec == MRTLBM_F64 ? "f64" : "f32")
      << (m->storage ? "m" : "d");
    return k.str();
}

extern "C" mrtlbm_status mrtlbm_autotune(mrtlbm_medium *m, const char *cache_path, mrtlbm_launch *best) {
    if (!m) return fail(MRTLBM_E_ARG, "medium is NULL");
    mrtlbm_status st = mrtlbm_init(m, nullptr, 0);
    if (st != MRTLBM_OK) return st;
    const double rs = (m->prec == MRTLBM_F64) ? 8.0 : 4.0;
    const double bytes_per_step = (double)m->N * (2.0 * mrtlbm_state_values(m) * rs + 1.0);
    long long n = (long long)std::ceil(2e10 / bytes_per_step);
    n = std::max(4LL, std::min(n, 2000LL));
    n += (n & 1);
    Launch bestL = m->launch;
    double bestms = 1e300;
    const Launch saved = m->launch;
    for (int vec : {4, 2, 1})
        for (int bx : {8, 16, 32, 64})
            for (int t : {64, 128, 256})
                for (int nt : {0, 1, 2, 3})
                    for (int map : {0, 1}) {
                Launch L{vec, bx, t / bx, nt, map};
                if (map && ((m->ny + L.by - 1) / L.by) % 8) continue;  // remap needs 8 | row blocks
                if (t % bx || !launch_ok(m, L)) continue;
                if (L.bx > 2 * std::max(8, m->nx / vec)) continue;  // mostly idle lanes
                m->launch = L;
                drop_graphs(m);
                double ms = 0;
                st = mrtlbm_time_steps(m, 2, &ms);  // warm-up
                if (st == MRTLBM_OK) st = mrtlbm_time_steps(m, n, &ms);
                if (st != MRTLBM_OK) {
                    m->launch = saved;
                    return st;
                }
                if (ms < bestms) {
                    bestms = ms;
                    bestL = L;
                }
            }
    m->launch = bestL;
    drop_graphs(m);
    m->initialised = false;
    if (best) {
        best->vec = bestL.vec; best->bx = bestL.bx; best->by = bestL.by; best->nt = bestL.nt; best->map = bestL.map;
    }
    if (cache_path) {
        const std::string key = tune_key(m);
        std::vector<std::string> lines;
        {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line))
                if (line.compare(0, key.size() + 1, key + " ") != 0 && !line.empty()) lines.push_back(line);
        }
        std::ostringstream l;
        l << key << ' ' << bestL.vec << ' ' << bestL.bx << ' ' << bestL.by << ' ' << bestL.nt << ' ' << bestL.map << ' '
          << (bestms / n);
        lines.push_back(l.str());
        std::ofstream o(cache_path, std::ios::trunc);
        for (auto &s : lines) o << s << '\n';
        if (!o) return fail(MRTLBM_E_ARG, "cannot write %s", cache_path);
    }
    return MRTLBM_OK;
}

extern "C" mrtlbm_status mrtlbm_load_tuned(mrtlbm_medium *m, const char *cache_path) {
    if (!m || !cache_path) return fail(MRTLBM_E_ARG, "NULL argument");
    const std::string key = tune_key(m);
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
        std::istringstream r(line.substr(key.size() + 1));
        Launch L{};
        if (r >> L.vec >> L.bx >> L.by >> L.nt >> L.map && launch_ok(m, L)) {
            drop_graphs(m);
            m->launch = L;
            return MRTLBM_OK;
        }
    }
    return MRTLBM_NOT_CONVERGED;
}
