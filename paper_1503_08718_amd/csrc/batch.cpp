// placeholder, replaced by the batched driver
#include "medium.h"
using namespace mrt;
extern "C" size_t mrtlbm_batch_workspace_bytes(mrtlbm_medium *const *, int) { return 0; }
extern "C" mrtlbm_status mrtlbm_batch_solve(mrtlbm_medium *const *, int, double, mrtlbm_tol_kind, long long, int,
                                            void *, size_t, mrtlbm_result *) {
    return fail(MRTLBM_E_ARG, "not built");
}
