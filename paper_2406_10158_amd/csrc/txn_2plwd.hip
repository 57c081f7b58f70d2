// Instantiation of the transaction kernel for one scheme (CC_2PL_WD), with
// latch-free or latched control-word updates.
#include "txn_kernel.h"

namespace cce {

hipError_t launch_txn_2plwd(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, bool strict, bool latch,
                           const RunArgs &a, int n_cu, int *grid_used) {
  if (latch)
    return strict ? dispatch<CC_2PL_WD, true, true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                  : dispatch<CC_2PL_WD, false, true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
  return strict ? dispatch<CC_2PL_WD, true, false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                : dispatch<CC_2PL_WD, false, false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
}

}  // namespace cce
