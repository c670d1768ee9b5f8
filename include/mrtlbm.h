/*
 * mrtlbm.h -- C ABI of the MI355X (gfx950) solver for steady anisotropic heat
 * conduction in voxelised heterogeneous media by the D3Q7 multiple-relaxation-
 * time lattice Boltzmann method of Fang, Gou, Zhang, Chen and Tao
 * ("Numerical predictions of effective thermal conductivities for 3D
 * four-directional braided composites using the lattice Boltzmann method").
 *
 * Conventions (every entry point):
 *   - Grids are [nz][ny][nx], x fastest.  Node (i, j, k) is the centre of voxel
 *     (i, j, k); phase interfaces and the outer walls lie on voxel faces, half
 *     way between nodes (the half lattice division of Sec. 2.3).
 *   - Pointers named *_dev are device pointers; *_host are host pointers.
 *     All device memory is owned by the caller (e.g. torch tensors): the phase
 *     grid, the workspace and every output.  The library owns only the opaque
 *     host-side medium, a 256-byte pinned host staging buffer and its graphs.
 *   - "real" means float for MRTLBM_F32 media and double for MRTLBM_F64 media.
 *   - All device work is enqueued on the stream given at creation (NULL = the
 *     default stream).  Calls that return host values synchronise that stream.
 *   - No exception or abort crosses the ABI.  Every call returns an
 *     mrtlbm_status (0 = OK, < 0 = error, > 0 = warning);
 *     mrtlbm_last_error() gives a message for the calling thread.
 *   - Lattice units: voxel edge = time step = 1.  A phase with physical
 *     conductivity tensor k gets the lattice diffusivity D = s k (Eq. 13 with
 *     rho c_p = 1 in every phase, Eq. 20), where one scale s per medium makes
 *     the largest eigenvalue of tau - I/2 over all phases equal dmax.
 *     Effective conductivities are returned in the units of k.
 *   - A medium is not thread-safe; distinct media are independent.
 */
#ifndef MRTLBM_H
#define MRTLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRTLBM_OK = 0,
    MRTLBM_NOT_CONVERGED = 1,   /* warning: max_steps ran out; results are valid partials */
    MRTLBM_E_ARG = -1,          /* bad argument, dims, phase id >= nphase, size mismatch  */
    MRTLBM_E_TENSOR = -2,       /* a conductivity tensor is not symmetric positive definite */
    MRTLBM_E_BC = -3,           /* bad boundary specification                             */
    MRTLBM_E_HIP = -4,          /* a HIP runtime call failed                              */
    MRTLBM_E_NONFINITE = -5,    /* the state holds NaN or Inf                             */
    MRTLBM_E_DIVERGED = -6,     /* the residual grew by > 1e3 across checks               */
    MRTLBM_E_WORKSPACE = -7     /* workspace too small or misaligned                      */
} mrtlbm_status;

typedef enum { MRTLBM_F32 = 0, MRTLBM_F64 = 1 } mrtlbm_precision;
typedef enum { MRTLBM_PERIODIC = 0, MRTLBM_ADIABATIC = 1 } mrtlbm_side;
typedef enum {
    MRTLBM_TOL_MAXDT = 0, /* stop when max |T(t) - T(t-1)| at a check < tol                        */
    MRTLBM_TOL_KEFF = 1   /* stop after two checks in a row at which: the energy balance
                             |k_hot - k_cold + k_side + k_leak| / k < tol; the volume-mean flux
                             agrees, |k_vol - k| / k < tol (skipped when side fluxes are set);
                             and the last change of k between checks, with its geometric tail,
                             is < tol/4 */
} mrtlbm_tol_kind;

typedef struct mrtlbm_medium mrtlbm_medium;

/*
 * Observables of one streaming step t -> t+1 (Eq. 22 evaluated three ways):
 *   keff_hot / keff_cold: wall link fluxes through the hot / cold Dirichlet
 *       face, N_g Phi / (dT A s), A = nodes per face;
 *   keff_vol: N_g <q_g> / (dT s), the volume mean of the node flux (Eqs.
 *       15-16) of the distribution arriving at t+1;
 *   keff = (keff_hot + keff_cold) / 2;
 *   keff_col[a] = N_g <q_a> / (dT s): the gradient column of the effective
 *       tensor (keff_col[grad_axis] == keff_vol);
 *   resid = max over nodes of |T(t+1) - T(t)|;
 *   temp_mean = mean T(t+1);
 *   keff_leak = N_g L / (dT A s), L the energy the rounding of this step
 *       added to the stored state (summed exactly in FP64); at steady state
 *       keff_hot - keff_cold + keff_leak = 0, and the MRTLBM_TOL_KEFF rule
 *       tests |keff_hot - keff_cold + keff_leak| / keff (the stored energy's
 *       rate of change), which equals the wall-flux gap in exact arithmetic,
 *       together with |keff_vol - keff| (transients that move heat inside
 *       the cell without changing its energy) and the change of keff;
 *   keff_side: the heat imposed through Neumann faces in the same units
 *       (0 unless mrtlbm_set_side_flux was called); at steady state
 *       keff_hot - keff_cold + keff_side + keff_leak = 0, and the rule
 *       includes it.  With side inflow the two wall fluxes differ and keff is
 *       only their mean, not a conductivity.
 */
typedef struct {
    double keff, keff_hot, keff_cold, keff_vol;
    double keff_col[3];
    double resid;
    double temp_mean;
    double keff_leak;
    double keff_side; /* heat imposed through Neumann faces (mrtlbm_set_side_flux), N_g sum(q A_f) / (dT A) */
    long long steps;  /* steps taken by the medium when the values were taken */
    int converged;
    int nonfinite;    /* nodes whose T(t+1) is not finite */
} mrtlbm_result;

/* Thread-block shape of the step kernel: each thread updates `vec`
 * consecutive x nodes; a block is bx x by threads over (x-vectors, rows).
 * vec in {1, 2, 4} (nx % vec == 0), bx in {8, 16, 32, 64}, bx*by in [64, 256]
 * and a multiple of 64, vec*bx >= 16.  nt: cache policy of the state
 * streams, bit 0 = non-temporal loads, bit 1 = non-temporal stores.  map = 1:
 * XCD-aware block order (each of the 8 XCDs sweeps one slab of rows through
 * all planes, so rows and planes pulled from neighbours are still in that
 * XCD's L2; used when the number of row blocks is a multiple of 8).
 * The batched solver uses vec, bx*by (threads per row tile) and nt of cells[0]. */
typedef struct { int vec, bx, by, nt, map; } mrtlbm_launch;

/* Bytes of caller-owned device workspace a medium of these sizes needs
 * (two state buffers of 7 reals per node, reduction partials and tables),
 * or 0 for invalid sizes.  Enough for either state storage.  Valid sizes:
 * nx, ny, nz >= 1 (an extent of 1 is allowed: the node is then its own
 * periodic neighbour, or lies on both walls of that axis), nz <= 65535,
 * ny <= 16 * 65535, 1 <= nphase <= 256. */
size_t mrtlbm_workspace_bytes(int nx, int ny, int nz, int nphase, mrtlbm_precision p);

/* The same for one state storage (0: 7 populations per node, 1: 4 moments
 * per node; see mrtlbm_set_storage), or 0 for invalid arguments.  A medium
 * created on a workspace of the storage-1 size starts in moment storage and
 * cannot switch to populations (E_WORKSPACE). */
size_t mrtlbm_workspace_bytes_storage(int nx, int ny, int nz, int nphase, mrtlbm_precision p, int storage);

/*
 * Create a medium (Sec. 2.2-2.3; Eqs. 12-13 for the per-phase tables).
 *   phase_dev: uint8 [nz][ny][nx]; borrowed, must outlive the medium; every
 *       id must be < nphase (checked on the device, MRTLBM_E_ARG otherwise).
 *   k_host: [nphase][6] = (kxx, kyy, kzz, kxy, kxz, kyz), physical units;
 *       copied.  Each tensor must be symmetric positive definite
 *       (MRTLBM_E_TENSOR).  1 <= nphase <= 256.
 *   workspace_dev: >= mrtlbm_workspace_bytes_storage(..., 1) bytes,
 *       256-byte aligned, caller-owned, must outlive the medium; the medium
 *       starts in population storage when the workspace holds it
 *       (>= mrtlbm_workspace_bytes), otherwise in moment storage.
 *   hip_stream: a hipStream_t, or NULL for the default stream.
 * Defaults: dmax = 1, gradient along x with T = 1 on the x = 0 face and
 * T = 0 on the far x face, periodic y and z, state not initialised.
 */
mrtlbm_status mrtlbm_create(int nx, int ny, int nz, const unsigned char *phase_dev,
                            const double *k_host, int nphase, mrtlbm_precision p,
                            void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                            mrtlbm_medium **out);

/* Boundary conditions (Sec. 2.3, Eqs. 23-25).  grad_axis (0, 1, 2) gets
 * isothermal walls: t_hot on its index-0 face and t_cold on its last face
 * (Eq. 23, half-way anti-bounce-back); t_hot != t_cold.  side[a] for the two
 * other axes: MRTLBM_PERIODIC (Eq. 25) or MRTLBM_ADIABATIC (Eq. 24 with zero
 * flux, half-way bounce-back); side[grad_axis] is ignored.  Invalidates the
 * state: call mrtlbm_init afterwards. */
mrtlbm_status mrtlbm_set_bc(mrtlbm_medium *m, int grad_axis, double t_hot, double t_cold,
                            const int side[3]);

/* Neumann faces with a given heat flux (Eq. 24): q_lo and q_hi are the heat
 * fluxes INTO the cell through the index-0 and the last face of `axis`, in
 * the units of mrtlbm_flux (k times temperature per voxel); each wall link
 * then re-enters with the reflected population plus s * q.  axis must be a
 * side with MRTLBM_ADIABATIC faces (E_BC otherwise); mrtlbm_set_bc resets
 * both to 0.  The state stays valid.  Errors: E_ARG (NULL, not finite), E_BC. */
mrtlbm_status mrtlbm_set_side_flux(mrtlbm_medium *m, int axis, double q_lo, double q_hi);

/* Relaxation times tau_4, tau_5, tau_6 of Eq. 12 (default 1, as the paper
 * sets them), one set for all phases; each must exceed 1/2.  Values other
 * than 1 need population storage (E_ARG under moment storage, and
 * mrtlbm_set_storage(m, 1) then fails) and are not accepted by
 * mrtlbm_batch_solve.  The step then relaxes all six non-conserved moments of
 * Eq. 11 (7 populations per node); in FP32 the seven outputs are formed
 * exactly in FP64 from the FP32 inputs and each is rounded to FP32 with the
 * dither described at mrtlbm_set_storage.  The state stays valid. */
mrtlbm_status mrtlbm_set_relaxation(mrtlbm_medium *m, double tau4, double tau5, double tau6);

/* Relaxation scale: largest eigenvalue of tau - I/2 over all phases
 * (Eq. 13; the paper keeps tau_ii in (0.5, 2)).  0 < dmax <= 1.5.
 * Invalidates the state. */
mrtlbm_status mrtlbm_set_scale(mrtlbm_medium *m, double dmax);

/* Initial state (Eq. 6): every node at equilibrium with temperature
 * t0_dev[z][y][x] (real), or with T = 0 if t0_dev is NULL.  With
 * flags & 1 the flux part of a non-equilibrium start is added from central
 * differences of t0 (Eq. 15 read backwards).  Resets the step counter. */
mrtlbm_status mrtlbm_init(mrtlbm_medium *m, const void *t0_dev, int flags);

/* Advance nsteps collide-and-stream steps (Eqs. 5, 8, 21, 23-25); async. */
mrtlbm_status mrtlbm_step(mrtlbm_medium *m, long long nsteps);

/*
 * Iterate to steady state.  Every check_every steps (even, >= 2) the last
 * step of the block evaluates the observables in FP64; the stop rule `kind`
 * is tested on them.  Returns MRTLBM_OK when converged,
 * MRTLBM_NOT_CONVERGED when max_steps ran out (out holds the last check),
 * MRTLBM_E_NONFINITE / MRTLBM_E_DIVERGED on failure.  Synchronises.
 */
mrtlbm_status mrtlbm_solve(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind, long long max_steps,
                           int check_every, mrtlbm_result *out);

/*
 * For callers that cannot allocate memory (serving loops and harnesses that
 * forbid hipMalloc and graph instantiation): mrtlbm_solve without hip graphs
 * (every step is its own launch) and with the check step's per-block
 * partials and final reduction in a fixed device array of the library
 * instead of the medium's workspace.  Same arguments, stop rules, return
 * values and results as mrtlbm_solve, bit for bit.  The array holds the
 * partials of up to 65536 check blocks (5.2 MB per device, kept until the
 * process ends); a medium whose check step needs more (a cross-section of
 * more than about 2^20 x-vectors of the launch shape) gets
 * MRTLBM_E_WORKSPACE before any device work.  Calls on the same device
 * share that array: calls that overlap in time on one device race and
 * must be serialised by the caller.  Synchronises.
 */
mrtlbm_status mrtlbm_solve_noalloc(mrtlbm_medium *m, double tol, mrtlbm_tol_kind kind, long long max_steps,
                                   int check_every, mrtlbm_result *out);

/* Observables of the next streaming step, computed without changing the
 * state (see mrtlbm_result).  Synchronises. */
mrtlbm_status mrtlbm_keff(mrtlbm_medium *m, mrtlbm_result *out);

/* Temperature T(t) = sum_i f_i (Eq. 14) into t_dev (real [nz][ny][nx]); async. */
mrtlbm_status mrtlbm_temperature(mrtlbm_medium *m, void *t_dev);

/* Node heat flux of the distribution arriving at t+1 (Eqs. 15-16, Fourier's
 * sign), q = -k grad T in units of k times temperature per voxel edge, into
 * q_dev (real [3][nz][ny][nx]); async. */
mrtlbm_status mrtlbm_flux(mrtlbm_medium *m, void *q_dev);

/* How the state is stored (Sec. 2.2: with tau_4 = tau_5 = tau_6 = 1 the
 * post-collision state of a node is fixed by four moments, T and
 * jhat = (I - tau^-1) j):
 *   0 (default): the seven post-collision populations minus w_i T_lin(x),
 *      real [7][nz][ny][nx] (T_lin: the linear profile between the walls);
 *   1: the moments (T - T_lin(x), jhat_x/2, jhat_y/2, jhat_z/2),
 *      real [4][nz][ny][nx]: 4 instead of 7 values per node and per step
 *      read and written.  In FP64 the populations are recomputed from them
 *      with the operations that produce them in storage 0, so both storages
 *      give bit-identical fields.  In FP32 they are recomputed exactly (in
 *      FP64), so a step rounds only the new T and jhat/2; storage 0 has to
 *      round each population and the two agree to FP32 noise.
 *   FP32 rounding (both storages) is dithered: values computed in FP64 are
 *      rounded up with probability equal to the discarded fraction, with
 *      random bits hashed from the value and the node, a deterministic
 *      function of the state.
 * Invalidates the state.  E_WORKSPACE when the workspace is too small for
 * the storage, E_ARG for storage 1 with tau_4..6 other than 1. */
mrtlbm_status mrtlbm_set_storage(mrtlbm_medium *m, int storage);

/* Values per node of the state: 7 (storage 0) or 4 (storage 1). */
int mrtlbm_state_values(const mrtlbm_medium *m);

/* Checkpoint / resume: copy the library's state (real [v][nz][ny][nx],
 * v = mrtlbm_state_values, layout as for mrtlbm_set_storage) out of or into
 * the medium, device to device, on the medium's stream.  A resumed medium
 * continues bit for bit.  state_set also sets the step counter. */
mrtlbm_status mrtlbm_state_get(mrtlbm_medium *m, void *f_dev);
mrtlbm_status mrtlbm_state_set(mrtlbm_medium *m, const void *f_dev, long long steps);

/* Scale s, steps taken, and the launch shape in use. */
mrtlbm_status mrtlbm_info(const mrtlbm_medium *m, double *scale, long long *steps, mrtlbm_launch *launch);

/* Choose the step kernel's block shape.  NULL restores the default. */
mrtlbm_status mrtlbm_set_launch(mrtlbm_medium *m, const mrtlbm_launch *launch);

/* Time every admissible block shape on this medium (hip events, a few
 * steps each), keep the fastest, and record it in the text file cache_path
 * (keyed by device architecture, sizes and precision; NULL = no file).
 * Clobbers the state: call before mrtlbm_init.  Synchronises. */
mrtlbm_status mrtlbm_autotune(mrtlbm_medium *m, const char *cache_path, mrtlbm_launch *best);

/* Look the block shape up in a cache written by mrtlbm_autotune; returns
 * MRTLBM_NOT_CONVERGED (a warning) and leaves the shape alone on a miss. */
mrtlbm_status mrtlbm_load_tuned(mrtlbm_medium *m, const char *cache_path);

/* Run nsteps plain steps bracketed by hip events on the medium's stream and
 * return the elapsed milliseconds.  Synchronises. */
mrtlbm_status mrtlbm_time_steps(mrtlbm_medium *m, long long nsteps, double *ms);

/* Measurement calibration, not part of the method: a plain streaming copy
 * of `streams` (1, 2, 4 or 7) separate arrays of n16 16-byte elements each,
 * src_dev[k][n16] -> dst_dev[k][n16], every lane issuing all its loads before
 * its stores; nt != 0 uses non-temporal loads and stores.  The step kernel
 * moves 4 (moment storage) or 7 (population storage) such state arrays; the
 * copy of the same number of arrays is the HBM ceiling its bandwidth is read
 * against, and a copy of known size calibrates the HBM byte counters.
 * Both arrays 16-byte aligned and device-resident; async on hip_stream. */
mrtlbm_status mrtlbm_stream_copy(const void *src_dev, void *dst_dev, long long n16, int streams, int nt,
                                 void *hip_stream);

void mrtlbm_destroy(mrtlbm_medium *m);
const char *mrtlbm_last_error(void);

/* Progress reports of long solves: when set, mrtlbm_solve and
 * mrtlbm_batch_solve call fn(message, user) from the calling thread at check
 * points, at most once every interval_s seconds.  NULL switches it off.
 * Process-wide. */
typedef void (*mrtlbm_progress_fn)(const char *message, void *user);
void mrtlbm_set_progress(mrtlbm_progress_fn fn, void *user, double interval_s);

/* ------------------------------------------------------------------------ */
/* Batched many-cell solver                                                  */
/* ------------------------------------------------------------------------ */

/* Bytes of device workspace mrtlbm_batch_solve needs for these media. */
size_t mrtlbm_batch_workspace_bytes(mrtlbm_medium *const *cells, int n);

/*
 * Solve n initialised media together.  Every step is one kernel launch that
 * covers all still-active cells (a table of row tiles: whole rows packed over
 * a tile's threads, or x-chunks of rows longer than that), and the steps between
 * checks are replayed as one hip graph; a cell leaves the table when its own
 * stop rule holds.  All cells must share the precision and the stream of
 * cells[0]; the step's shape (vec, bx * by threads per row tile, nt, map)
 * is cells[0]'s launch shape (see mrtlbm_batch_autotune).  out: [n].
 * Returns MRTLBM_OK when every cell converged,
 * MRTLBM_NOT_CONVERGED if any ran out of steps.  Synchronises.
 */
mrtlbm_status mrtlbm_batch_solve(mrtlbm_medium *const *cells, int n, double tol, mrtlbm_tol_kind kind,
                                 long long max_steps, int check_every, void *workspace_dev,
                                 size_t workspace_bytes, mrtlbm_result *out);

/*
 * Pick the batched step's shape for exactly this set of media: times every
 * valid (vec, threads per row tile in {64, 128, 256}, cache policy nt, tile
 * order map) on all cells together, from zero states, over about 2e10
 * algorithmic bytes each, and stores the fastest in cells[0]'s launch shape,
 * which mrtlbm_batch_solve uses (map = 1: each XCD sweeps one contiguous
 * eighth of the tile table).  Overwrites the states: every cell is left
 * uninitialised with its step counter at 0, so call it before mrtlbm_init.
 * Same requirements and workspace as mrtlbm_batch_solve.  best may be NULL.
 * Synchronises.
 */
mrtlbm_status mrtlbm_batch_autotune(mrtlbm_medium *const *cells, int n, void *workspace_dev,
                                    size_t workspace_bytes, mrtlbm_launch *best);

#ifdef __cplusplus
}
#endif
#endif /* MRTLBM_H */
