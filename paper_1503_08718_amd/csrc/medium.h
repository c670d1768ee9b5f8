// Host-side state of one medium (the opaque mrtlbm_medium of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/mrtlbm.h"
#include "lbm_internal.h"

namespace mrt {

struct GraphEntry {
    int K;
    int cur;
    bool check;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct StopState {
    double kprev = 0.0, dprev = 0.0;
    bool have_prev = false, have_d = false;
    double min_resid = -1.0;
    int passes = 0;          // consecutive checks that met the k_eff rule
    bool check_vol = true;   // compare the volume-mean flux (off with imposed side fluxes)
};

mrtlbm_status fail(mrtlbm_status st, const char *fmt, ...);
// rate-limited progress report through the callback set by mrtlbm_set_progress
void progress(const char *fmt, ...);
mrtlbm_status hip_fail(hipError_t e, const char *what);
size_t partial_capacity(int nx, int ny);
// symmetric 3x3 helpers: (xx, yy, zz, xy, xz, yz) -> row-major 3x3; its
// eigenvalues (trigonometric solution of the cubic); positive definiteness
void sym_full(const double *k6, double *m);
void sym_eig(const double *m, double ev[3]);
bool sym_pd(const double *m);

}  // namespace mrt

struct mrtlbm_medium {
    int nx = 0, ny = 0, nz = 0;
    long long N = 0;
    int nphase = 0;
    mrtlbm_precision prec = MRTLBM_F32;
    const unsigned char *phase = nullptr;
    std::vector<double> k;          // [nphase][6], physical
    std::vector<double> tab_host;   // [nphase][TABW]
    std::vector<float> tab_host_f;
    double dmax = 1.0, s = 0.0;
    int gaxis = 0;
    double t_hot = 1.0, t_cold = 0.0;
    int side[3] = {0, 0, 0};
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *bufA = nullptr, *bufB = nullptr, *tab = nullptr;
    double *partials = nullptr, *final8 = nullptr;
    size_t pcap = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double *pinned = nullptr;  // host staging for reductions
    int device = 0;
    int cur = 0;               // state in bufA (0) or bufB (1)
    int storage = 0;           // 0: 7 populations per node, 1: 4 moments per node
    double tau_rest[3] = {1.0, 1.0, 1.0};  // tau_4, tau_5, tau_6 (Eq. 12)
    double qside[3][2] = {{0, 0}, {0, 0}, {0, 0}};  // imposed inflow on Neumann faces (physical)
    long long steps = 0;
    bool initialised = false;
    mrt::Launch launch{4, 64, 4, 0, 0};
    std::vector<mrt::GraphEntry> graphs;
};

namespace mrt {
bool launch_ok(const mrtlbm_medium *m, const Launch &L);
Launch default_launch(const mrtlbm_medium *m);
template <typename real>
Cell<real> make_cell(const mrtlbm_medium *m, int cur);
void drop_graphs(mrtlbm_medium *m);
void fill_result(const mrtlbm_medium *m, const double *f, mrtlbm_result *out);
int stop_rule(StopState &ss, const mrtlbm_result &r, double tol, mrtlbm_tol_kind kind);
bool has_side_flux(const mrtlbm_medium *m);
}  // namespace mrt
