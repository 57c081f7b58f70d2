// Instantiation of the transaction kernel for one scheme (CC_OCC), with
// latch-free or latched control-word updates, and of OCC's hot-row engine.
#include "hot_engine.h"
#include "txn_kernel.h"

namespace cce {

hipError_t launch_txn_occ(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, bool strict, bool latch,
                         const RunArgs &a, int n_cu, int *grid_used) {
  if (latch)
    return strict ? dispatch<CC_OCC, true, true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                  : dispatch<CC_OCC, false, true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
  return strict ? dispatch<CC_OCC, true, false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                : dispatch<CC_OCC, false, false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
}

hipError_t launch_engine_occ(hipStream_t s, int lanes, int max_ops, int waves, bool strict, const RunArgs &a,
                             const EngineArgs &e, int *threads_used) {
  return strict ? engine_dispatch<true>(s, lanes, max_ops, waves, a, e, threads_used)
                : engine_dispatch<false>(s, lanes, max_ops, waves, a, e, threads_used);
}

}  // namespace cce
