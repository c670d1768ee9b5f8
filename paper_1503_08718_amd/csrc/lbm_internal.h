// Internal interface between the host driver (api.cpp, batch.cpp) and the
// device code (lbm_kernels.hip, batch_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrt {

constexpr int Q = 7;
constexpr int NRED = 10;  // reduced quantities per partial (see RedIdx)
constexpr int TABW = 12; // table reals per phase: half (I - tau^-1) [6], tau - I [6]

enum RedIdx { R_PHI_HOT = 0, R_PHI_COLD, R_QX, R_QY, R_QZ, R_RESID, R_TSUM, R_NONFINITE, R_LEAK, R_SPARE };

// Per-medium geometry and boundary description passed to every kernel.
// The state is stored as g_i = f_hat_i - w_i T_lin(x): the post-collision
// distribution minus the equilibrium of the linear wall-to-wall profile.
template <typename real>
struct Cell {
    const real *src;          // state at t, [7][N]
    real *dst;                // state at t+1, [7][N]
    const uint8_t *phase;     // [N]
    const real *tab;          // [nphase][TABW]
    int nx, ny, nz, nxv;      // nxv = nx / vec
    long long N;              // nodes = population stride
    int nphase;
    int per[3];               // axis is periodic
    real sgn[3];              // reflection sign on a wall: -1 isothermal, +1 adiabatic
    real h[3];                // shift of the gradient-axis populations (eps dT / (2 N_g)), else 0
    int gaxis;
    int storage;              // 0: 7 populations [7][N]; 1: moments (T - T_lin, jhat/2) [4][N]
    int relax;                // 1: tau_4..6 not all 1 (population storage only)
    real srel[3];             // 1 / tau_4, 1 / tau_5, 1 / tau_6
    real phi[3][2];           // lattice heat inflow per link on the low / high face (Neumann), else 0
};

struct Launch {
    int vec, bx, by;
    int nt;   // bit 0: non-temporal state loads, bit 1: non-temporal state stores
    int map;  // 1: XCD-aware block order (each XCD sweeps one slab of rows)
};

// kernel launchers (lbm_kernels.hip)
template <typename real>
hipError_t launch_step(const Cell<real> &c, const Launch &L, hipStream_t s);

// mode 1: step + FP64 observables; mode 2: observables only (state unchanged);
// mode 3: as 2 and also write the node flux field q_out ([3][N], scaled by qscale)
template <typename real>
hipError_t launch_check(const Cell<real> &c, const Launch &L, int mode, double *partials, int *nblocks_out,
                        real *q_out, double qscale, hipStream_t s);
template <typename real>
int check_blocks(const Cell<real> &c, const Launch &L);

hipError_t launch_reduce(const double *partials, int nparts, double *final8, hipStream_t s);

template <typename real>
hipError_t launch_init(const Cell<real> &c, real *state, const real *t0, int flags, double t_hot, double dT,
                       hipStream_t s);
template <typename real>
hipError_t launch_temperature(const Cell<real> &c, const real *state, real *t_out, double t_hot, double dT,
                              hipStream_t s);
hipError_t launch_phase_max(const uint8_t *phase, long long n, int *block_max, int nblocks, hipStream_t s);

}  // namespace mrt
