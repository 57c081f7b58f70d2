// HIP kernels of the batch transaction engine (gfx950 / CDNA4, wave64).
//
// Execution model.  A 64-lane wavefront is split into teams of L lanes
// (L = 1, 4, 16 or 64); a team executes one transaction at a time, lane j of
// the team owning the transaction's operations j, j+L, j+2L, ... in
// registers (K slots per lane).  This replaces the paper's "warp density"
// knob -- 2^wd working threads per 32-lane warp, one transaction each
// (Section 4.1, "Launch Parameters") -- which on a 64-lane wavefront would
// leave lanes idle: here every lane works, and L trades lanes per transaction
// against transactions per wavefront.  Teams are persistent: a team takes the
// next transaction index from a device counter (one atomic per wavefront for
// all teams that need work), runs it until it commits -- restarting at once
// after an abort, as in the paper's procedure (Section 4.1, "Experimental
// Procedure") but after a short randomised back-off -- and takes the next.
//
// Memory ordering.  Every access to shared state (control words and table
// values) is an agent-scope atomic: loads and stores carry the device-scope
// coherence bit and read-modify-writes execute at the coherent cache level,
// so values written on one XCD are seen by the others.  Where a step must
// complete before the next starts (e.g. a row's version word is read before
// its value, a value is stored before the version word that publishes it) an
// ordering point waits for all outstanding memory operations of the
// wavefront; with CC_RUN_STRICT_FENCES it is a full agent-scope fence.  This
// replaces the paper's "volatile read + relaxed CAS + fence" recipe for
// latch-free critical sections (Section 3.4, "Atomic Operation").
#include "device.h"

namespace cce {

// ---------------------------------------------------------------------------
// Between passes: the list of transactions still pending (not committed, not
// given up), appended with one atomic per wavefront; order is irrelevant.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) pass_reset_kernel(Ctl *ctl) {
  if (threadIdx.x == 0) {
    ctl->queue = 0;
    ctl->pending_n = 0;
  }
}

__global__ void __launch_bounds__(256) compact_kernel(const DevOutcome *out, uint64_t n, uint64_t max_attempts,
                                                      uint32_t *list, Ctl *ctl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool p = false;
  if (i < n) {
    const DevOutcome o = out[i];
    p = o.status != CC_COMMITTED && o.attempts < max_attempts;
  }
  const uint64_t m = ballot(p);
  if (m == 0) return;
  const int lane = __lane_id();
  const int first = __ffsll((unsigned long long)m) - 1;
  uint64_t base = 0;
  if (lane == first) base = atomicAdd((unsigned long long *)&ctl->pending_n, (unsigned long long)__popcll(m));
  base = readlane64(base, first);
  if (p) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)i;
}

hipError_t launch_compact(hipStream_t s, const DevOutcome *out, uint64_t n_txns, uint64_t max_attempts,
                          uint32_t *list, Ctl *ctl) {
  hipLaunchKernelGGL(pass_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
  const uint64_t blocks = (n_txns + 255) / 256;
  if (blocks) hipLaunchKernelGGL(compact_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, n_txns, max_attempts,
                                 list, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CC initialisation: clear control words, outcomes and the control block.
// A plain fill kernel (not hipMemsetAsync) so that it can be graph-captured.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) init_kernel(uint64_t *words, uint64_t n_words, uint64_t *aux,
                                                   uint64_t n_aux, DevOutcome *out, uint64_t n_out, Ctl *ctl,
                                                   uint64_t ticket_start) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = tid; i < n_words; i += stride) words[i] = 0;
  for (uint64_t i = tid; i < n_aux; i += stride) aux[i] = 0;
  for (uint64_t i = tid; i < n_out; i += stride) {
    DevOutcome o;
    o.status = CC_PENDING;
    o.attempts = 0;
    o.serial_hi = 0;
    o.serial_lo = 0;
    o.commit_ns = -1;
    out[i] = o;
  }
  if (tid == 0) {
    ctl->queue = 0;
    ctl->ticket = ticket_start;
    ctl->pending_n = 0;
    ctl->budget_reserved = 0;
    ctl->budget_released = 0;
    for (int i = 0; i < DS_N; ++i) ctl->stats[i] = 0;
    ctl->stop = 0;
    ctl->start_clock = wall_clock64();
  }
}

hipError_t launch_init(hipStream_t s, uint64_t *words, uint64_t n_words, uint64_t *aux, uint64_t n_aux,
                       DevOutcome *out, uint64_t n_out, Ctl *ctl, uint64_t ticket_start) {
  uint64_t n = n_words > n_aux ? n_words : n_aux;
  n = n > n_out ? n : n_out;
  uint64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, n_words, aux, n_aux, out, n_out,
                     ctl, ticket_start);
  return hipGetLastError();
}

hipError_t launch_txn(hipStream_t s, int scheme, int lanes, int max_ops, int waves_per_wg, int grid, bool strict,
                      bool latch, const RunArgs &a, int n_cu, int *grid_used) {
  switch (scheme) {
    case CC_OCC: return launch_txn_occ(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    case CC_2PL_NW: return launch_txn_2pl(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    case CC_TO: return launch_txn_to(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    case CC_MVCC: return launch_txn_mvcc(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    case CC_TICTOC: return launch_txn_tictoc(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    case CC_2PL_WD: return launch_txn_2plwd(s, lanes, max_ops, waves_per_wg, grid, strict, latch, a, n_cu, grid_used);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cce
