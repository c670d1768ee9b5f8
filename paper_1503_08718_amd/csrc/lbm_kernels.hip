// Device code of the D3Q7 MRT lattice Boltzmann solver for gfx950.
//
// One step (Eqs. 5, 8, 21, 23-25), fused per node x:
//   pull   f_i(x) = g_i(x - e_i) from the state at t (Eq. 21; periodic wrap,
//          Eq. 25), or on a wall link the reflected local population,
//          f_i(x) = sgn * g_ibar(x) (Eq. 23 with sgn = -1, Eq. 24 with sgn = +1),
//          then add +-h on the gradient-axis pair;
//   collide with tau_0 = tau_4 = tau_5 = tau_6 = 1 (Sec. 2.2 sets them to unity):
//          the moments of Eq. 11 relax to (T, jhat, 3T/4, 0, 0) with
//          jhat = (I - tau^-1) j, so the post-collision state is
//          g_0 = T/4 and g_{2a+1,2a+2} = T/8 +- jhat_a / 2;
//   push   the 7 outputs to the state at t+1.
// g_i = f_hat_i - w_i T_lin(x) is the post-collision distribution minus the
// equilibrium of the linear profile T_lin between the two isothermal walls.
// The scheme is linear and P w = w, so this shift is exact: interior
// streaming along the gradient axis gains +-w dT/N_g = +-h and the wall
// terms eps (T_w - T_lin(node)) of Eq. 23 become +-h as well.  The stored
// numbers are deviations from a known field, which keeps FP32 round-off
// relative to the (small) deviation and flux rather than to T itself.
//
// Memory layout: structure of arrays, population-major [7][nz][ny][nx], x
// fastest.  Every population value is pulled by exactly one node, so a step
// reads 7 reals + 1 phase byte and writes 7 reals per node, each once.
// A thread owns `VEC` consecutive x nodes of one row: all 7 streams are
// aligned vector loads/stores, and the two x-moving populations take their
// single out-of-vector element from the neighbouring lane (ds_bpermute), so no
// unaligned access is issued.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_internal.h"

namespace mrt {

// Single-cell grid: a block is bx x by threads; the bx threads of a block row
// form a chunk of one lattice row, aligned inside a wave (bx divides 64).
template <int VEC, typename real>
__device__ __forceinline__ XLink chunk_links(const Cell<real> &c, int xv, int tx, int bx) {
    const int lane = __lane_id();
    XLink xl;
    const bool whole_row = (c.nxv <= bx);
    if (xv > 0) { xl.srcL = lane - 1; xl.haveL = tx > 0; }
    else { xl.srcL = lane + c.nxv - 1; xl.haveL = whole_row; }
    if (xv < c.nxv - 1) { xl.srcR = lane + 1; xl.haveR = tx < bx - 1; }
    else { xl.srcR = lane - (c.nxv - 1); xl.haveR = whole_row; }
    return xl;
}

// Block coordinates.  With MAP the linear dispatch order (workgroups go to
// the 8 XCDs round robin) is remapped so that each XCD sweeps one slab of
// y-blocks through all planes: the rows and planes a block pulls from its
// neighbours were then loaded by the same XCD moments before and are still in
// its L2 (requires gridDim.y % 8 == 0).
template <int MAP>
__device__ __forceinline__ void block_coords(int &bxi, int &byi, int &bzi) {
    if constexpr (MAP) {
        const unsigned gx = gridDim.x, gy = gridDim.y;
        const unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const unsigned slab = gy / 8, xcd = b % 8, seq = b / 8;
        bxi = (int)(seq % gx);
        const unsigned r = seq / gx;
        byi = (int)(xcd * slab + r % slab);
        bzi = (int)(r / slab);
    } else {
        bxi = blockIdx.x;
        byi = blockIdx.y;
        bzi = blockIdx.z;
    }
}

template <typename real, int VEC, int NT, int ST, int MAP>
__global__ void __launch_bounds__(256) k_step(Cell<real> c) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *tab = reinterpret_cast<real *>(smem_raw);
    // moment storage: the state loads go out before the table is staged
    // (measured faster there; population storage stages the table first)
    constexpr bool LATE_TABLE = (ST == 1);
    // moment storage: issue this wave's loads at raised priority; the pull
    // lowers it once they are all out (measured 0.7 us faster per FP32 step
    // at 256^3, 4.6 us per FP64 step)
    if constexpr (ST == 1) __builtin_amdgcn_s_setprio(3);
    TablePrefetch<real> tp;
    if constexpr (LATE_TABLE) tp = table_prefetch(c);
    else load_table(c, tab);
    int bxi, byi, bzi;
    block_coords<MAP>(bxi, byi, bzi);
    const int tx = threadIdx.x, bx = blockDim.x;
    int xv = bxi * bx + tx;
    int y = byi * blockDim.y + threadIdx.y;
    const int z = bzi;
    const bool active = (xv < c.nxv) && (y < c.ny);
    xv = min(xv, c.nxv - 1);
    y = min(y, c.ny - 1);
    Acc dummy;
    node_update<real, VEC, 0, NT, ST>(c, tab, xv, y, z, active, chunk_links<VEC>(c, xv, tx, bx), dummy, nullptr,
                                      real(0), [&](const real *&) {
                                          if constexpr (LATE_TABLE) table_commit(c, tab, tp);
                                      });
}

// Observables (and optionally the step): the grid covers x and y like the
// step kernel; each block walks `zper` consecutive planes so that the number
// of partials stays small and the summation order is fixed.
template <typename real, int VEC, int MODE, int ST>
__global__ void __launch_bounds__(256) k_check(Cell<real> c, int zper, double *partials, real *qout, real qscale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *tab = reinterpret_cast<real *>(smem_raw);
    load_table(c, tab);
    const int tx = threadIdx.x, bx = blockDim.x;
    int xv = blockIdx.x * bx + tx;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    const bool active = (xv < c.nxv) && (y < c.ny);
    xv = min(xv, c.nxv - 1);
    y = min(y, c.ny - 1);
    Acc acc;
    acc.zero();
    const int z0 = blockIdx.z * zper, z1 = min(c.nz, z0 + zper);
    const XLink xl = chunk_links<VEC>(c, xv, tx, bx);
    for (int z = z0; z < z1; z++) node_update<real, VEC, MODE, 0, ST>(c, tab, xv, y, z, active, xl, acc, qout, qscale);
    const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_reduce_store(acc, partials + b * NRED);
}

__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ partials, int nparts, double *final8) {
    __shared__ double red[256][NRED];
    const int t = threadIdx.x;
    double v[NRED];
    for (int k = 0; k < NRED; k++) v[k] = 0.0;
    for (int i = t; i < nparts; i += 256)
        for (int k = 0; k < NRED; k++) {
            double p = partials[(long long)i * NRED + k];
            v[k] = (k == R_RESID) ? fmax(v[k], p) : v[k] + p;
        }
    for (int k = 0; k < NRED; k++) red[t][k] = v[k];
    __syncthreads();
    for (int stride = 128; stride >= 1; stride >>= 1) {
        if (t < stride)
            for (int k = 0; k < NRED; k++)
                red[t][k] = (k == R_RESID) ? fmax(red[t][k], red[t + stride][k]) : red[t][k] + red[t + stride][k];
        __syncthreads();
    }
    if (t < NRED) final8[t] = red[0][t];
}

// T_lin at node index i of the gradient axis: walls at -1/2 and n - 1/2
__device__ __forceinline__ double t_lin(int i, int n, double t_hot, double dT) {
    return t_hot - (i + 0.5) * dT / n;
}

template <typename real>
__global__ void k_init(Cell<real> c, real *state, const real *t0, int flags, double t_hot, double dT) {
    const long long n = c.N;
    const int ext[3] = {c.nx, c.ny, c.nz};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % c.nx);
        const long long r = i / c.nx;
        const int y = (int)(r % c.ny), z = (int)(r / c.ny);
        const int pos[3] = {x, y, z};
        const int g = c.gaxis;
        const double tl = t_lin(pos[g], ext[g], t_hot, dT);
        const double T = t0 ? (double)t0[i] : 0.0;
        const double dev = T - tl;
        double jh[3] = {0.0, 0.0, 0.0};
        if ((flags & 1) && t0) {
            // grad T by central differences; walls: isothermal value at the
            // half-way plane, adiabatic mirror, periodic wrap
            double grad[3];
            const long long stride[3] = {1, c.nx, (long long)c.nx * c.ny};
            for (int a = 0; a < 3; a++) {
                double lo, hi, dist = 2.0;
                const int p = pos[a];
                if (p > 0) lo = t0[i - stride[a]];
                else if (c.per[a]) lo = t0[i + (long long)(ext[a] - 1) * stride[a]];
                else if (a == g) { lo = t_hot; dist -= 0.5; }
                else lo = T;
                if (p < ext[a] - 1) hi = t0[i + stride[a]];
                else if (c.per[a]) hi = t0[i - (long long)(ext[a] - 1) * stride[a]];
                else if (a == g) { hi = t_hot - dT; dist -= 0.5; }
                else hi = T;
                grad[a] = (hi - lo) / dist;
            }
            // pre-collision j = -eps tau grad T (Eq. 15); jhat = (I - tau^-1) j
            // = -eps (tau - I) grad T
            const real *tb = c.tab + c.phase[i] * TABW + 6;  // tau - I
            const double m[3][3] = {{tb[0], tb[3], tb[4]}, {tb[3], tb[1], tb[5]}, {tb[4], tb[5], tb[2]}};
            for (int a = 0; a < 3; a++) jh[a] = -0.25 * (m[a][0] * grad[0] + m[a][1] * grad[1] + m[a][2] * grad[2]);
        }
        // round the moments (T - T_lin, jhat / 2) once to the storage
        // precision; the populations are built from those rounded moments
        // exactly as a collision builds them, so both storages start alike
        const real Tr = (real)dev;
        if (c.storage) {
            state[i] = Tr;
            for (int a = 0; a < 3; a++) state[(a + 1) * n + i] = (real)(0.5 * jh[a]);
        } else {
            state[i] = Tr * real(0.25);
            for (int a = 0; a < 3; a++) {
                const real zr = (real)(0.5 * jh[a]);
                state[(2 * a + 1) * n + i] = gplus(Tr, zr);
                state[(2 * a + 2) * n + i] = gminus(Tr, zr);
            }
        }
    }
}

template <typename real>
__global__ void k_temperature(Cell<real> c, const real *__restrict__ state, real *__restrict__ t_out, double t_hot,
                              double dT) {
    const long long n = c.N;
    const int ext[3] = {c.nx, c.ny, c.nz};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % c.nx);
        const long long r = i / c.nx;
        const int pos[3] = {x, (int)(r % c.ny), (int)(r / c.ny)};
        // T = sum of the seven populations, in the same order for both
        // storages (moment storage rebuilds each population first)
        real acc;
        if (!c.storage) {
            acc = state[i];
            for (int q = 1; q < Q; q++) acc += state[q * n + i];
        } else {
            const real T = state[i];
            acc = T * real(0.25);
            for (int a = 1; a < 4; a++) {
                const real z = state[a * n + i];
                acc += gplus(T, z);
                acc += gminus(T, z);
            }
        }
        t_out[i] = (real)((double)acc + t_lin(pos[c.gaxis], ext[c.gaxis], t_hot, dT));
    }
}

__global__ void k_phase_max(const uint8_t *__restrict__ phase, long long n, int *block_max) {
    __shared__ int red[256];
    int m = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        m = max(m, (int)phase[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static inline dim3 step_grid(int nxv, int ny, int nz, const Launch &L) {
    return dim3((nxv + L.bx - 1) / L.bx, (ny + L.by - 1) / L.by, nz);
}

template <typename real, int ST, int MAP>
static void launch_step_st(const Cell<real> &cc, const Launch &L, dim3 grid, dim3 block, size_t sh, hipStream_t s) {
    switch (L.vec * 4 + (L.nt & 3)) {
        case 16: hipLaunchKernelGGL((k_step<real, 4, 0, ST, MAP>), grid, block, sh, s, cc); break;
        case 17: hipLaunchKernelGGL((k_step<real, 4, 1, ST, MAP>), grid, block, sh, s, cc); break;
        case 18: hipLaunchKernelGGL((k_step<real, 4, 2, ST, MAP>), grid, block, sh, s, cc); break;
        case 19: hipLaunchKernelGGL((k_step<real, 4, 3, ST, MAP>), grid, block, sh, s, cc); break;
        case 8: hipLaunchKernelGGL((k_step<real, 2, 0, ST, MAP>), grid, block, sh, s, cc); break;
        case 9: hipLaunchKernelGGL((k_step<real, 2, 1, ST, MAP>), grid, block, sh, s, cc); break;
        case 10: hipLaunchKernelGGL((k_step<real, 2, 2, ST, MAP>), grid, block, sh, s, cc); break;
        case 11: hipLaunchKernelGGL((k_step<real, 2, 3, ST, MAP>), grid, block, sh, s, cc); break;
        case 4: hipLaunchKernelGGL((k_step<real, 1, 0, ST, MAP>), grid, block, sh, s, cc); break;
        case 5: hipLaunchKernelGGL((k_step<real, 1, 1, ST, MAP>), grid, block, sh, s, cc); break;
        case 6: hipLaunchKernelGGL((k_step<real, 1, 2, ST, MAP>), grid, block, sh, s, cc); break;
        default: hipLaunchKernelGGL((k_step<real, 1, 3, ST, MAP>), grid, block, sh, s, cc); break;
    }
}

template <typename real>
hipError_t launch_step(const Cell<real> &c, const Launch &L, hipStream_t s) {
    Cell<real> cc = c;
    cc.nxv = c.nx / L.vec;
    const dim3 grid = step_grid(cc.nxv, c.ny, c.nz, L), block(L.bx, L.by);
    const size_t sh = sizeof(real) * TABW * c.nphase;
    const bool map = L.map && (grid.y % 8 == 0);
    if (cc.storage) {
        if (map) launch_step_st<real, 1, 1>(cc, L, grid, block, sh, s);
        else launch_step_st<real, 1, 0>(cc, L, grid, block, sh, s);
    } else if (cc.relax) {
        if (map) launch_step_st<real, 2, 1>(cc, L, grid, block, sh, s);
        else launch_step_st<real, 2, 0>(cc, L, grid, block, sh, s);
    } else {
        if (map) launch_step_st<real, 0, 1>(cc, L, grid, block, sh, s);
        else launch_step_st<real, 0, 0>(cc, L, grid, block, sh, s);
    }
    return hipGetLastError();
}

static inline int check_zper(int gx, int gy, int nz) {
    const long long xy = (long long)gx * gy;
    long long zb = (2048 + xy - 1) / xy;  // aim at ~2048 blocks
    if (zb > nz) zb = nz;
    if (zb < 1) zb = 1;
    return (int)((nz + zb - 1) / zb);
}

template <typename real>
int check_blocks(const Cell<real> &c, const Launch &L) {
    const int nxv = c.nx / L.vec;
    const dim3 g = step_grid(nxv, c.ny, c.nz, L);
    const int zper = check_zper(g.x, g.y, c.nz);
    return g.x * g.y * ((c.nz + zper - 1) / zper);
}

template <typename real, int VEC, int ST>
static void launch_check_st(const Cell<real> &c, dim3 grid, dim3 block, size_t sh, int zper, int mode, double *parts,
                            real *q, real qs, hipStream_t s) {
    switch (mode) {
        case 1: hipLaunchKernelGGL((k_check<real, VEC, 1, ST>), grid, block, sh, s, c, zper, parts, q, qs); break;
        case 2: hipLaunchKernelGGL((k_check<real, VEC, 2, ST>), grid, block, sh, s, c, zper, parts, q, qs); break;
        default: hipLaunchKernelGGL((k_check<real, VEC, 3, ST>), grid, block, sh, s, c, zper, parts, q, qs); break;
    }
}

template <typename real, int VEC>
static void launch_check_vec(const Cell<real> &c, dim3 grid, dim3 block, size_t sh, int zper, int mode, double *parts,
                             real *q, real qs, hipStream_t s) {
    if (c.storage) launch_check_st<real, VEC, 1>(c, grid, block, sh, zper, mode, parts, q, qs, s);
    else if (c.relax) launch_check_st<real, VEC, 2>(c, grid, block, sh, zper, mode, parts, q, qs, s);
    else launch_check_st<real, VEC, 0>(c, grid, block, sh, zper, mode, parts, q, qs, s);
}

template <typename real>
hipError_t launch_check(const Cell<real> &c, const Launch &L, int mode, double *partials, int *nblocks_out, real *q_out,
                        double qscale, hipStream_t s) {
    Cell<real> cc = c;
    cc.nxv = c.nx / L.vec;
    const dim3 g = step_grid(cc.nxv, c.ny, c.nz, L);
    const int zper = check_zper(g.x, g.y, c.nz);
    const dim3 grid(g.x, g.y, (c.nz + zper - 1) / zper), block(L.bx, L.by);
    const size_t sh = sizeof(real) * TABW * c.nphase;
    if (nblocks_out) *nblocks_out = grid.x * grid.y * grid.z;
    switch (L.vec) {
        case 4: launch_check_vec<real, 4>(cc, grid, block, sh, zper, mode, partials, q_out, (real)qscale, s); break;
        case 2: launch_check_vec<real, 2>(cc, grid, block, sh, zper, mode, partials, q_out, (real)qscale, s); break;
        default: launch_check_vec<real, 1>(cc, grid, block, sh, zper, mode, partials, q_out, (real)qscale, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nparts, double *final8, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nparts, final8);
    return hipGetLastError();
}

static inline int grid_1d(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

template <typename real>
hipError_t launch_init(const Cell<real> &c, real *state, const real *t0, int flags, double t_hot, double dT,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_init<real>), dim3(grid_1d(c.N)), dim3(256), 0, s, c, state, t0, flags, t_hot, dT);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_temperature(const Cell<real> &c, const real *state, real *t_out, double t_hot, double dT,
                              hipStream_t s) {
    hipLaunchKernelGGL((k_temperature<real>), dim3(grid_1d(c.N)), dim3(256), 0, s, c, state, t_out, t_hot, dT);
    return hipGetLastError();
}

hipError_t launch_phase_max(const uint8_t *phase, long long n, int *block_max, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_phase_max, dim3(nblocks), dim3(256), 0, s, phase, n, block_max);
    return hipGetLastError();
}

#define MRT_INST(real)                                                                                             \
    template hipError_t launch_step<real>(const Cell<real> &, const Launch &, hipStream_t);                        \
    template hipError_t launch_check<real>(const Cell<real> &, const Launch &, int, double *, int *, real *, double, \
                                           hipStream_t);                                                           \
    template int check_blocks<real>(const Cell<real> &, const Launch &);                                           \
    template hipError_t launch_init<real>(const Cell<real> &, real *, const real *, int, double, double, hipStream_t); \
    template hipError_t launch_temperature<real>(const Cell<real> &, const real *, real *, double, double,          \
                                                 hipStream_t);
MRT_INST(float)
MRT_INST(double)

}  // namespace mrt
