// Internal interface of the batched many-cell step (batch_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace mrt {

// tiles: int4 (cell, z-plane, first row, number of rows); one block each.
// chunk > 0: XCD-aware order over a table of 8 * chunk tiles (padded with
// empty tiles); partials are indexed by tile.
template <typename real>
hipError_t launch_batch(const Cell<real> *cells, const int4 *tiles, int ntiles, int vec, int threads, int max_nphase,
                        int parity, bool check, int nt, int chunk, int storage, double *partials, hipStream_t s);

// finals[c][8] = fixed-order reduction of partials[start[c] .. start[c+1])
hipError_t launch_batch_reduce(const double *partials, const int *start, int ncells, double *finals, hipStream_t s);

}  // namespace mrt
