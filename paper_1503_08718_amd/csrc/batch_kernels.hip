// Batched step over many cells in one launch.
//
// Every block takes one "row tile" from a table: a run of whole lattice rows
// (x lines) of one z-plane of one cell.  The cell's descriptor supplies its
// sizes, boundaries, buffers and phase table, so cells of different size,
// braiding angle and yarn fraction share a launch.  A thread owns `VEC`
// consecutive nodes of one row; the rows of a tile are packed back to back
// over the block's threads (a row may straddle two waves, in which case the
// x-neighbour element at the seam is loaded instead of shuffled).  The
// per-node arithmetic is the single-cell kernel's (node_update), so a batched
// cell evolves bit for bit like the same cell stepped alone.
#include <hip/hip_runtime.h>

#include "batch_internal.h"
#include "lbm_device.hpp"

namespace mrt {

__device__ __forceinline__ XLink packed_links(int xv, int nxv) {
    const int lane = __lane_id();
    XLink xl;
    if (xv > 0) { xl.srcL = lane - 1; xl.haveL = lane > 0; }
    else { xl.srcL = lane + nxv - 1; xl.haveL = lane + nxv - 1 <= 63; }
    if (xv < nxv - 1) { xl.srcR = lane + 1; xl.haveR = lane < 63; }
    else { xl.srcR = lane - (nxv - 1); xl.haveR = lane - (nxv - 1) >= 0; }
    return xl;
}

// tile = (cell, z-plane, first row y0, number of rows), or for rows longer
// than the block (cell, z-plane, row, -1 - x-chunk).  chunk > 0: the
// table holds 8 * chunk tiles and block b takes tile (b % 8) * chunk + b / 8,
// so that each XCD (blocks go to the 8 XCDs round robin) sweeps one
// contiguous eighth of the table and finds the neighbouring rows and planes
// it pulls in its own L2.
template <typename real, int VEC, int MODE, int NT, int ST>
__global__ void __launch_bounds__(256) k_batch(const Cell<real> *__restrict__ cells, const int4 *__restrict__ tiles,
                                               int parity, int chunk, double *partials) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *tab = reinterpret_cast<real *>(smem_raw);
    const int ti = chunk ? (int)(blockIdx.x % 8u) * chunk + (int)(blockIdx.x / 8u) : (int)blockIdx.x;
    const int4 tile = tiles[ti];
    Cell<real> c = cells[tile.x];
    if (parity) {
        const real *t = c.src;
        c.src = c.dst;
        c.dst = const_cast<real *>(t);
    }
    load_table(c, tab);
    const int t = threadIdx.x;
    int xv, y;
    bool active;
    if (tile.w >= 0) {  // tile.w whole rows from tile.z
        const int rows = blockDim.x / c.nxv;
        const int r = t / c.nxv;
        xv = t - r * c.nxv;
        y = tile.z + r;
        active = (r < rows) && (r < tile.w) && (y < c.ny);
    } else {  // x-chunk -1 - tile.w of row tile.z
        xv = (-1 - tile.w) * (int)blockDim.x + t;
        y = tile.z;
        active = xv < c.nxv;
    }
    xv = min(xv, c.nxv - 1);
    y = min(y, c.ny - 1);
    const int z = tile.y;
    Acc acc;
    acc.zero();
    node_update<real, VEC, MODE, NT, ST>(c, tab, xv, y, z, active, packed_links(xv, c.nxv), acc, nullptr, real(0));
    if constexpr (MODE == 1) block_reduce_store(acc, partials + (long long)ti * NRED);
}

// one block per cell: fixed-order sum of that cell's tile partials
__global__ void __launch_bounds__(256) k_batch_reduce(const double *__restrict__ partials, const int *__restrict__ start,
                                                      double *__restrict__ finals) {
    __shared__ double red[256][NRED];
    const int cell = blockIdx.x, t = threadIdx.x;
    const int b = start[cell], e = start[cell + 1];
    double v[NRED];
    for (int k = 0; k < NRED; k++) v[k] = 0.0;
    for (int i = b + t; i < e; i += 256)
        for (int k = 0; k < NRED; k++) {
            const double p = partials[(long long)i * NRED + k];
            v[k] = (k == R_RESID) ? fmax(v[k], p) : v[k] + p;
        }
    for (int k = 0; k < NRED; k++) red[t][k] = v[k];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (t < s)
            for (int k = 0; k < NRED; k++)
                red[t][k] = (k == R_RESID) ? fmax(red[t][k], red[t + s][k]) : red[t][k] + red[t + s][k];
        __syncthreads();
    }
    if (t < NRED) finals[(long long)cell * NRED + t] = red[0][t];
}

template <typename real, int VEC, int ST>
static void launch_batch_st(const Cell<real> *cells, const int4 *tiles, int ntiles, int threads, size_t sh, int parity,
                            bool check, int nt, int chunk, double *partials, hipStream_t s) {
    const dim3 g(ntiles), b(threads);
    if (check) hipLaunchKernelGGL((k_batch<real, VEC, 1, 0, ST>), g, b, sh, s, cells, tiles, parity, chunk, partials);
    else if (nt == 3)
        hipLaunchKernelGGL((k_batch<real, VEC, 0, 3, ST>), g, b, sh, s, cells, tiles, parity, chunk, partials);
    else if (nt == 2)
        hipLaunchKernelGGL((k_batch<real, VEC, 0, 2, ST>), g, b, sh, s, cells, tiles, parity, chunk, partials);
    else if (nt == 1)
        hipLaunchKernelGGL((k_batch<real, VEC, 0, 1, ST>), g, b, sh, s, cells, tiles, parity, chunk, partials);
    else hipLaunchKernelGGL((k_batch<real, VEC, 0, 0, ST>), g, b, sh, s, cells, tiles, parity, chunk, partials);
}

template <typename real, int VEC>
static void launch_batch_vec(const Cell<real> *cells, const int4 *tiles, int ntiles, int threads, size_t sh, int parity,
                             bool check, int nt, int chunk, int storage, double *partials, hipStream_t s) {
    if (storage) launch_batch_st<real, VEC, 1>(cells, tiles, ntiles, threads, sh, parity, check, nt, chunk, partials, s);
    else launch_batch_st<real, VEC, 0>(cells, tiles, ntiles, threads, sh, parity, check, nt, chunk, partials, s);
}

template <typename real>
hipError_t launch_batch(const Cell<real> *cells, const int4 *tiles, int ntiles, int vec, int threads, int max_nphase,
                        int parity, bool check, int nt, int chunk, int storage, double *partials, hipStream_t s) {
    const size_t sh = sizeof(real) * TABW * max_nphase;
    switch (vec) {
        case 4:
            launch_batch_vec<real, 4>(cells, tiles, ntiles, threads, sh, parity, check, nt, chunk, storage, partials, s);
            break;
        case 2:
            launch_batch_vec<real, 2>(cells, tiles, ntiles, threads, sh, parity, check, nt, chunk, storage, partials, s);
            break;
        default:
            launch_batch_vec<real, 1>(cells, tiles, ntiles, threads, sh, parity, check, nt, chunk, storage, partials, s);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const double *partials, const int *start, int ncells, double *finals, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reduce, dim3(ncells), dim3(256), 0, s, partials, start, finals);
    return hipGetLastError();
}

template hipError_t launch_batch<float>(const Cell<float> *, const int4 *, int, int, int, int, int, bool, int, int, int,
                                        double *, hipStream_t);
template hipError_t launch_batch<double>(const Cell<double> *, const int4 *, int, int, int, int, int, bool, int, int,
                                         int, double *, hipStream_t);

}  // namespace mrt
