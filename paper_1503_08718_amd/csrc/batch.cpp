// Batched many-cell driver: all still-active cells advance together, one
// kernel launch per step over a table of row tiles, the steps between two
// checks replayed as one hip graph; a cell leaves the table when its own stop
// rule holds (the same rule as mrtlbm_solve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "batch_internal.h"
#include "medium.h"

using namespace mrt;

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct BatchLayout {
    size_t cells, tiles, partials, start, finals, total;
    long long max_tiles;
};

bool batch_layout(mrtlbm_medium *const *cells, int n, BatchLayout *L) {
    if (!cells || n < 1) return false;
    long long mt = 0;
    for (int i = 0; i < n; i++) {
        if (!cells[i]) return false;
        // rows of up to 64 threads' worth of nodes per tile at the least
        // (vec 1, 64 threads): enough for every shape the batch may take
        mt += (long long)cells[i]->nz * cells[i]->ny * ((cells[i]->nx + 63) / 64);
    }
    mt += 8;  // room to pad the table to a multiple of 8 (XCD-aware order)
    if (mt > (1LL << 31) - 1) return false;
    size_t o = 0;
    L->cells = o; o = align256(o + (size_t)n * sizeof(Cell<double>));
    L->tiles = o; o = align256(o + (size_t)mt * sizeof(int4));
    L->partials = o; o = align256(o + (size_t)mt * NRED * sizeof(double));
    L->start = o; o = align256(o + (size_t)(n + 1) * sizeof(int));
    L->finals = o; o = align256(o + (size_t)n * NRED * sizeof(double));
    L->total = o;
    L->max_tiles = mt;
    return true;
}

struct BatchRun {
    mrtlbm_medium *const *cells = nullptr;
    int n = 0;
    int vec = 1, threads = 256, max_nphase = 1, nt = 0, storage = 0;
    int map = 0;    // XCD-aware tile order
    int chunk = 0;  // tiles per XCD when map is set
    char *ws = nullptr;
    BatchLayout lay{};
    hipStream_t stream = nullptr, cap = nullptr;  // cap is owned (destroyed with the run)
    double *pinned = nullptr;
    std::vector<int> active;  // indices into cells
    int ntiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~BatchRun() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (pinned) (void)hipHostFree(pinned);
    }
};

template <typename real>
mrtlbm_status upload_cells(BatchRun &B) {
    std::vector<Cell<real>> desc(B.n);
    for (int i = 0; i < B.n; i++) {
        desc[i] = make_cell<real>(B.cells[i], B.cells[i]->cur);
        desc[i].nxv = B.cells[i]->nx / B.vec;
    }
    hipError_t e = hipMemcpyAsync(B.ws + B.lay.cells, desc.data(), desc.size() * sizeof(Cell<real>),
                                  hipMemcpyHostToDevice, B.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "batch cell table upload");
}

// tiles of the active cells (contiguous per cell) and per-cell tile ranges.
// A tile is (cell, z, y0, rows): `rows` whole rows from y0, packed over the
// block's threads; a row longer than the block is cut into x-chunks of one
// tile each, (cell, z, y, -1 - chunk).
mrtlbm_status upload_tiles(BatchRun &B) {
    std::vector<int4> tiles;
    std::vector<int> start;
    for (int a : B.active) {
        const mrtlbm_medium *m = B.cells[a];
        const int nxv = m->nx / B.vec;
        start.push_back((int)tiles.size());
        if (nxv <= B.threads) {
            const int rows = B.threads / nxv;
            for (int z = 0; z < m->nz; z++)
                for (int y0 = 0; y0 < m->ny; y0 += rows) tiles.push_back(int4{a, z, y0, std::min(rows, m->ny - y0)});
        } else {
            const int chunks = (nxv + B.threads - 1) / B.threads;
            for (int z = 0; z < m->nz; z++)
                for (int y = 0; y < m->ny; y++)
                    for (int k = 0; k < chunks; k++) tiles.push_back(int4{a, z, y, -1 - k});
        }
    }
    start.push_back((int)tiles.size());
    B.chunk = 0;
    if (B.map) {
        // pad with empty tiles (no rows: every thread inactive) to 8 * chunk
        while (tiles.size() % 8) tiles.push_back(int4{B.active.empty() ? 0 : B.active[0], 0, 0, 0});
        B.chunk = (int)(tiles.size() / 8);
    }
    B.ntiles = (int)tiles.size();
    if ((long long)B.ntiles > B.lay.max_tiles) return fail(MRTLBM_E_WORKSPACE, "tile table overflow");
    hipError_t e = hipMemcpyAsync(B.ws + B.lay.tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice,
                                  B.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.ws + B.lay.start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, B.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "batch tile table upload");
}

template <typename real>
mrtlbm_status build_graph(BatchRun &B, int K) {
    if (B.exec) { (void)hipGraphExecDestroy(B.exec); B.exec = nullptr; }
    if (B.graph) { (void)hipGraphDestroy(B.graph); B.graph = nullptr; }
    const Cell<real> *cells = (const Cell<real> *)(B.ws + B.lay.cells);
    const int4 *tiles = (const int4 *)(B.ws + B.lay.tiles);
    double *partials = (double *)(B.ws + B.lay.partials);
    const int *start = (const int *)(B.ws + B.lay.start);
    double *finals = (double *)(B.ws + B.lay.finals);
    hipError_t e = hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    for (int i = 0; i < K && e == hipSuccess; i++)
        e = launch_batch<real>(cells, tiles, B.ntiles, B.vec, B.threads, B.max_nphase, i & 1, i == K - 1, B.nt,
                               B.chunk, B.storage, partials, B.cap);
    if (e == hipSuccess) e = launch_batch_reduce(partials, start, (int)B.active.size(), finals, B.cap);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.pinned, finals, B.active.size() * NRED * sizeof(double), hipMemcpyDeviceToHost, B.cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(B.cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "batch graph capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    B.graph = g;
    e = hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "batch graph instantiate");
}

template <typename real>
mrtlbm_status run(BatchRun &B, double tol, mrtlbm_tol_kind kind, long long max_steps, int K, mrtlbm_result *out) {
    mrtlbm_status st = upload_cells<real>(B);
    if (st != MRTLBM_OK) return st;
    std::vector<StopState> ss(B.n);
    for (int i = 0; i < B.n; i++) ss[i].check_vol = !has_side_flux(B.cells[i]);
    std::vector<int> state(B.n, 0);  // 0 active, 1 converged, 2 out of steps, -1 non-finite, -2 diverged
    for (int i = 0; i < B.n; i++) {
        std::vector<double> zero(NRED, 0.0);
        fill_result(B.cells[i], zero.data(), &out[i]);
        if (B.cells[i]->steps + K <= max_steps) B.active.push_back(i);
        else state[i] = 2;
    }
    bool rebuild = true;
    while (!B.active.empty()) {
        if (rebuild) {
            st = upload_tiles(B);
            if (st == MRTLBM_OK) st = build_graph<real>(B, K);
            if (st != MRTLBM_OK) return st;
            rebuild = false;
        }
        hipError_t e = hipGraphLaunch(B.exec, B.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(B.stream);
        if (e != hipSuccess) return hip_fail(e, "batch graph launch");
        std::vector<int> still;
        for (size_t k = 0; k < B.active.size(); k++) {
            const int i = B.active[k];
            mrtlbm_medium *m = B.cells[i];
            m->steps += K;
            fill_result(m, B.pinned + k * NRED, &out[i]);
            const int v = stop_rule(ss[i], out[i], tol, kind);
            if (v == 1) { out[i].converged = 1; state[i] = 1; }
            else if (v < 0) state[i] = v;
            else if (m->steps + K > max_steps) state[i] = 2;
            else still.push_back(i);
        }
        progress("batch: %zu of %d cells still active after this check (%d tiles)", still.size(), B.n, B.ntiles);
        if (still.size() != B.active.size()) rebuild = true;
        B.active.swap(still);
    }
    int worst = 0;
    for (int i = 0; i < B.n; i++) {
        if (state[i] == -1) return fail(MRTLBM_E_NONFINITE, "cell %d became non-finite", i);
        if (state[i] == -2) worst = -2;
        if (state[i] == 2 && worst == 0) worst = 2;
    }
    if (worst == -2) return fail(MRTLBM_E_DIVERGED, "a cell diverged");
    return worst == 2 ? MRTLBM_NOT_CONVERGED : MRTLBM_OK;
}

// checks shared by the batched solve and its autotuner; fills B
static mrtlbm_status prepare(BatchRun &B, mrtlbm_medium *const *cells, int n, void *workspace_dev,
                             size_t workspace_bytes, bool need_init) {
    BatchLayout lay;
    if (!batch_layout(cells, n, &lay)) return fail(MRTLBM_E_ARG, "bad cell list");
    if (!workspace_dev || workspace_bytes < lay.total)
        return fail(MRTLBM_E_WORKSPACE, "batch workspace of %zu bytes, need %zu", workspace_bytes, lay.total);
    if (((uintptr_t)workspace_dev) & 255) return fail(MRTLBM_E_WORKSPACE, "workspace not 256-byte aligned");
    const mrtlbm_medium *m0 = cells[0];
    int vec = m0->launch.vec, threads = m0->launch.bx * m0->launch.by, max_nphase = 1;
    for (int i = 0; i < n; i++) {
        const mrtlbm_medium *m = cells[i];
        if (need_init && !m->initialised) return fail(MRTLBM_E_ARG, "cell %d is not initialised", i);
        if (m->prec != m0->prec) return fail(MRTLBM_E_ARG, "cells mix precisions");
        if (m->storage != m0->storage) return fail(MRTLBM_E_ARG, "cells mix state storages");
        if (m->tau_rest[0] != 1.0 || m->tau_rest[1] != 1.0 || m->tau_rest[2] != 1.0)
            return fail(MRTLBM_E_ARG, "batched solves need tau_4 = tau_5 = tau_6 = 1 (cell %d)", i);
        if (m->stream != m0->stream || m->device != m0->device) return fail(MRTLBM_E_ARG, "cells mix streams/devices");
        while (m->nx % vec) vec >>= 1;
        max_nphase = std::max(max_nphase, m->nphase);
        for (int j = 0; j < i; j++)
            if (cells[j] == m) return fail(MRTLBM_E_ARG, "cell %d listed twice", i);
    }
    if (vec < 1) vec = 1;
    // rows longer than a tile's threads are cut into x-chunks (one tile per
    // chunk of one row)
    B.cells = cells;
    B.n = n;
    B.vec = vec;
    B.threads = threads;
    B.max_nphase = max_nphase;
    B.nt = m0->launch.nt;
    B.map = m0->launch.map;
    B.storage = m0->storage;
    B.ws = (char *)workspace_dev;
    B.lay = lay;
    B.stream = m0->stream;
    B.cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void **)&B.pinned, (size_t)n * NRED * sizeof(double), hipHostMallocDefault);
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "batch setup");
}

// time `steps` (even) batched steps of all cells in the shape held by B
template <typename real>
static mrtlbm_status time_batch(BatchRun &B, int steps, double *ms) {
    if (B.active.empty()) return fail(MRTLBM_E_ARG, "no cells to time");
    mrtlbm_status st = upload_cells<real>(B);
    if (st == MRTLBM_OK) st = upload_tiles(B);
    if (st != MRTLBM_OK) return st;
    const Cell<real> *cells = (const Cell<real> *)(B.ws + B.lay.cells);
    const int4 *tiles = (const int4 *)(B.ws + B.lay.tiles);
    double *partials = (double *)(B.ws + B.lay.partials);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    for (int i = 0; i < 2 && e == hipSuccess; i++)  // warm-up
        e = launch_batch<real>(cells, tiles, B.ntiles, B.vec, B.threads, B.max_nphase, i & 1, false, B.nt, B.chunk,
                               B.storage, partials, B.stream);
    if (e == hipSuccess) e = hipEventRecord(a, B.stream);
    for (int i = 0; i < steps && e == hipSuccess; i++)
        e = launch_batch<real>(cells, tiles, B.ntiles, B.vec, B.threads, B.max_nphase, i & 1, false, B.nt, B.chunk,
                               B.storage, partials, B.stream);
    if (e == hipSuccess) e = hipEventRecord(b, B.stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float f = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *ms = f;
    return e == hipSuccess ? MRTLBM_OK : hip_fail(e, "batch timing");
}

}  // namespace

extern "C" size_t mrtlbm_batch_workspace_bytes(mrtlbm_medium *const *cells, int n) {
    BatchLayout L;
    return batch_layout(cells, n, &L) ? L.total : 0;
}

extern "C" mrtlbm_status mrtlbm_batch_solve(mrtlbm_medium *const *cells, int n, double tol, mrtlbm_tol_kind kind,
                                            long long max_steps, int check_every, void *workspace_dev,
                                            size_t workspace_bytes, mrtlbm_result *out) {
    if (!out) return fail(MRTLBM_E_ARG, "out is NULL");
    if (check_every < 2 || (check_every & 1)) return fail(MRTLBM_E_ARG, "check_every must be even and >= 2");
    if (!(tol > 0)) return fail(MRTLBM_E_ARG, "tol must be > 0");
    if (kind != MRTLBM_TOL_MAXDT && kind != MRTLBM_TOL_KEFF) return fail(MRTLBM_E_ARG, "bad tolerance kind");
    BatchRun B;
    mrtlbm_status st = prepare(B, cells, n, workspace_dev, workspace_bytes, true);
    if (st != MRTLBM_OK) return st;
    return cells[0]->prec == MRTLBM_F64 ? run<double>(B, tol, kind, max_steps, check_every, out)
                                        : run<float>(B, tol, kind, max_steps, check_every, out);
}

extern "C" mrtlbm_status mrtlbm_batch_autotune(mrtlbm_medium *const *cells, int n, void *workspace_dev,
                                               size_t workspace_bytes, mrtlbm_launch *best) {
    BatchRun B;
    mrtlbm_status st = prepare(B, cells, n, workspace_dev, workspace_bytes, false);
    if (st != MRTLBM_OK) return st;
    for (int i = 0; i < n; i++) {
        st = mrtlbm_init(cells[i], nullptr, 0);
        if (st != MRTLBM_OK) return st;
        B.active.push_back(i);
    }
    double bytes = 0.0;
    const double rs = cells[0]->prec == MRTLBM_F64 ? 8.0 : 4.0;
    for (int i = 0; i < n; i++) bytes += (double)cells[i]->N * (2.0 * mrtlbm_state_values(cells[i]) * rs + 1.0);
    int steps = (int)std::ceil(2e10 / bytes);
    steps = std::max(4, std::min(steps, 2000));
    steps += steps & 1;
    double bestms = 1e300;
    int bv = B.vec, bt = B.threads, bn = B.nt, bm = B.map;
    for (int vec : {4, 2, 1})
        for (int threads : {64, 128, 256})
            for (int nt : {0, 1, 2, 3})
                for (int map : {0, 1}) {
                    bool ok = true;
                    for (int i = 0; i < n && ok; i++)
                        ok = cells[i]->nx % vec == 0;
                    if (!ok) continue;
                    B.vec = vec; B.threads = threads; B.nt = nt; B.map = map;
                    double ms = 0.0;
                    st = cells[0]->prec == MRTLBM_F64 ? time_batch<double>(B, steps, &ms)
                                                      : time_batch<float>(B, steps, &ms);
                    if (st != MRTLBM_OK) return st;
                    if (ms < bestms) { bestms = ms; bv = vec; bt = threads; bn = nt; bm = map; }
                }
    // the batched solve takes vec, bx * by, nt and map from cells[0]
    mrtlbm_medium *m0 = cells[0];
    const int bx = std::min(bt, 64);
    m0->launch = Launch{bv, bx, bt / bx, bn, bm};
    drop_graphs(m0);
    for (int i = 0; i < n; i++) {
        cells[i]->initialised = false;
        cells[i]->steps = 0;
    }
    if (best) { best->vec = bv; best->bx = bx; best->by = bt / bx; best->nt = bn; best->map = bm; }
    progress("batch autotune: vec %d, %d threads per tile, nt %d, map %d: %.3f ms per step", bv, bt, bn, bm,
             bestms / steps);
    return MRTLBM_OK;
}
