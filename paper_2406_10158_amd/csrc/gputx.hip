// GPUTx (conflict-graph ordering by K-sets), a deterministic scheme.  The
// paper's description (Section 2, "Conflict Graph Ordering"): conflicts
// between transactions form a DAG ordered by transaction id; each
// transaction gets a rank from it, transactions of one rank (a K-set) run
// together without concurrency control, and the K-sets run in rank order.
// The rank here is the transaction's level in the DAG: one more than the
// largest rank among the earlier transactions it conflicts with (read-write,
// write-read, write-write on one item), 0 if none -- the rank that makes
// every K-set conflict-free.
//
// gfx950 design (preprocessing shared with GaccO, gacco.hip):
//  1. access table, radix sort by row, lock table: every row gets a turn
//     counter and every row access its place in the row's id-ordered list;
//  2. rank pass (gputx_rank_kernel): persistent teams take transactions in
//     id order; once every row of a transaction has come to it, the team
//     reads each row's state -- the largest rank of any earlier accessor and
//     the rank of the last earlier writer, both kept +1 in one 64-bit word --
//     takes the transaction's rank as the largest "one more than what it
//     conflicts with", updates the rows' states and passes the rows on;
//  3. stable radix sort of (rank, transaction) pairs, and the first
//     position of every rank (gputx_kstart_kernel);
//  4. execution (gputx_exec_kernel): persistent teams take sorted positions
//     in order; a position runs once every transaction of a lower rank is
//     done (one done counter), its operations as plain loads and stores --
//     no other transaction of its K-set touches its rows -- and the team
//     adds itself to the done counter after its stores are performed.
// Waiting, in both passes, is a state of the team in the persistent loop
// (never a spin) for transactions taken earlier by running wavefronts, so
// the smallest unfinished one can always proceed; a team that sees no
// progress for the wait limit stops the run (a safeguard, as for GaccO).
#include "opset.h"
#include "txn_kernel.h"

namespace cce {

__global__ void __launch_bounds__(64) gputx_reset_kernel(Ctl *ctl) {
  if (threadIdx.x == 0) {
    ctl->queue = 0;   // claim counter of the next pass
    ctl->ticket = 0;  // execution: transactions done
  }
}

__global__ void __launch_bounds__(256) gputx_fill_kernel(uint64_t *p, uint64_t n, uint32_t *iota, uint64_t n_iota) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i < n_iota) iota[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// rank pass
// ---------------------------------------------------------------------------
// Packed state (PACKED, batches of fewer than 2^20 transactions and 2^24
// operations): a row's word holds its turn and its state together --
// [63:40] place in the row's list whose turn it is, [39:20] largest rank + 1
// of its accessors so far, [19:0] rank + 1 of its last writer.  The look that
// finds the turn brings the state with it, and one store passes the row on
// with its new state, so neither a separate load of the state nor an
// ordering point before the release is needed.  Otherwise the state lives in
// its own word (kstate) and the turn word holds sorted positions.
constexpr uint64_t GX_M20 = (1ull << 20) - 1;

template <int L, int K, bool STRICT, bool PACKED>
__global__ void __launch_bounds__(MaxThreads<K>::value) gputx_rank_kernel(GputxArgs a) {
  constexpr int NW = L == 64 ? K : 1;
  static_assert(L == 64 || L * K <= 64, "operation sets of one word");
  using Set = OpSet<NW>;
  Team<L> t;
  int64_t txn = -1;
  bool finished = false;
  uint32_t rowk[K], rk[K];
  uint64_t gst[K];  // PACKED: the row's word as seen when its turn came
  Set lead = Set::zero(), granted = Set::zero();
  uint64_t ready_at = 0, progress_at = 0;
  uint32_t idle_polls = 0;

  for (;;) {
    const bool need = txn < 0 && !finished;
    const uint64_t q = t.claim(&a.ctl->queue, need, 1);
    bool fresh = false;
    if (need) {
      if (q < a.n_txns && ld_word(&a.ctl->stop) == 0) {
        txn = (int64_t)q;
        fresh = true;
      } else {
        finished = true;
      }
    }
    if (ballot(txn >= 0) == 0) break;
    const uint64_t now = wall_clock64();
    if (ballot(fresh)) {
      uint32_t first = 0, n = 0;
      if (fresh) {
        const DevTxn d = a.txns[txn];
        first = d.first;
        n = d.n;
      }
      bool ld[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
        ld[k] = false;
        if (fresh && idx < n) {
          const uint32_t r = a.ops[first + idx].rowk;
          ld[k] = op_leader(r);
          if (ld[k]) {
            rowk[k] = r;
            rk[k] = a.rank[first + idx];
          }
        }
      }
      const Set sl = team_set<L, K, NW>(t, ld);
      if (fresh) {
        lead = sl;
        granted = Set::zero();
        ready_at = 0;
        progress_at = now;
        idle_polls = 0;
      }
    }
    const bool act = txn >= 0 && now >= ready_at;
    bool g[K];
    uint64_t ahead = ~0ull;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t i = (uint32_t)t.tl + (uint32_t)(k * L);
      g[k] = false;
      if (act && lead.test(i) && !granted.test(i)) {
        const uint64_t w = ld_word(a.words + op_row(rowk[k]));
        const uint64_t turn = PACKED ? (w >> 40) : w;
        g[k] = turn == (uint64_t)rk[k];
        if (PACKED && g[k]) gst[k] = w;
        if (!g[k] && (uint64_t)rk[k] > turn) {
          const uint64_t d = (uint64_t)rk[k] - turn;
          ahead = d < ahead ? d : ahead;
        }
      }
    }
    const Set newly = team_set<L, K, NW>(t, g);
    if (act) granted = granted | newly;
    // every row has come to the transaction: its rank, the rows' new states,
    // then the rows move on
    const bool ready = act && granted == lead;
    if (PACKED && ballot(ready)) {
      uint64_t r1 = 1;  // the transaction's rank + 1: at least 1, else the largest of these
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (ready && lead.test((uint32_t)t.tl + (uint32_t)(k * L))) {
          const uint64_t any1 = (gst[k] >> 20) & GX_M20, w1 = gst[k] & GX_M20;
          const uint64_t c = op_written(rowk[k]) ? any1 + 1 : w1 + 1;
          r1 = c > r1 ? c : r1;
        }
      }
      r1 = t.max(r1);
      if (STRICT) order_point<STRICT>();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (ready && lead.test((uint32_t)t.tl + (uint32_t)(k * L))) {
          const uint64_t any1 = (gst[k] >> 20) & GX_M20, w1 = gst[k] & GX_M20;
          const uint64_t nany = any1 > r1 ? any1 : r1;
          const uint64_t nw1 = op_written(rowk[k]) ? r1 : w1;
          st_word(a.words + op_row(rowk[k]), (((uint64_t)rk[k] + 1) << 40) | (nany << 20) | nw1);
        }
      }
      if (ready && t.tl == 0) a.txn_rank[txn] = (uint32_t)(r1 - 1);
    } else if (!PACKED && ballot(ready)) {
      if (STRICT) order_point<STRICT>();
      else asm volatile("" ::: "memory");
      uint64_t st[K];
      uint64_t r1 = 1;  // the transaction's rank + 1: at least 1, else the largest of these
#pragma unroll
      for (int k = 0; k < K; ++k) {
        st[k] = 0;
        if (ready && lead.test((uint32_t)t.tl + (uint32_t)(k * L))) {
          st[k] = ld_word(a.kstate + op_row(rowk[k]));
          const uint64_t c = op_written(rowk[k]) ? (st[k] >> 32) + 1 : (st[k] & 0xFFFFFFFFull) + 1;
          r1 = c > r1 ? c : r1;
        }
      }
      r1 = t.max(r1);  // rank + 1 (at least 1)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (ready && lead.test((uint32_t)t.tl + (uint32_t)(k * L))) {
          const uint64_t any1 = (st[k] >> 32) > r1 ? (st[k] >> 32) : r1;
          const uint64_t w1 = op_written(rowk[k]) ? r1 : (st[k] & 0xFFFFFFFFull);
          st_word(a.kstate + op_row(rowk[k]), (any1 << 32) | w1);
        }
      }
      order_point<STRICT>();  // the rows' states are performed before the rows move on
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (ready && lead.test((uint32_t)t.tl + (uint32_t)(k * L)))
          st_word(a.words + op_row(rowk[k]), (uint64_t)rk[k] + 1);
      if (ready && t.tl == 0) a.txn_rank[txn] = (uint32_t)(r1 - 1);
    }
    if (txn >= 0) {
      const uint64_t after = wall_clock64();
      if (ready) {
        txn = -1;
      } else if (act && !(newly == Set::zero())) {
        progress_at = after;
        idle_polls = 0;
      } else {
        const uint64_t m = ~t.max(~ahead);  // team minimum of `ahead`
        if (act) {
          if (m != ~0ull && m > 1) {
            const uint64_t cap = 4096ull * a.poll_ticks;
            const uint64_t nap = (m - 1) * a.poll_ticks;
            ready_at = after + (nap < cap ? nap : cap);
          }
          ++idle_polls;
        }
        if (after - progress_at > a.wait_limit_ticks) {
          st_word(&a.ctl->stop, 1);
          finished = true;
          txn = -1;
        } else if ((idle_polls & 255u) == 255u && ld_word(&a.ctl->stop) != 0) {
          finished = true;
          txn = -1;
        }
      }
    }
    if (ballot(act) == 0) __builtin_amdgcn_s_sleep(2);
  }
}

// first sorted position of every rank
__global__ void __launch_bounds__(256) gputx_kstart_kernel(const uint32_t *rank_sorted, uint64_t n, uint32_t *kstart) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rank_sorted[i];
  if (r < n && (i == 0 || rank_sorted[i - 1] != r)) kstart[r] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// execution, K-set by K-set
// ---------------------------------------------------------------------------
template <int L, int K, bool STRICT>
__global__ void __launch_bounds__(MaxThreads<K>::value) gputx_exec_kernel(GputxArgs a) {
  Team<L> t;
  const uint64_t start_clock = a.ctl->start_clock;
  int64_t pos = -1;  // sorted position the team runs (team-uniform)
  bool finished = false;
  uint32_t txn = 0, need = 0;
  uint64_t ready_at = 0, progress_at = 0, began = 0, waited = 0;
  uint32_t idle_polls = 0;
  uint64_t n_commit = 0, t_useful = 0, t_wait = 0;
  bool staged = false;        // the claimed transaction's operations are in registers
  uint32_t first = 0, n = 0;
  uint32_t rowk[K], elem[K];
  int64_t arg[K];

  for (;;) {
    const bool claim = pos < 0 && !finished;
    const uint64_t q = t.claim(&a.ctl->queue, claim, 1);
    if (claim) {
      if (q < a.n_txns && ld_word(&a.ctl->stop) == 0) {
        pos = (int64_t)q;
        txn = a.order[q];
        need = a.kstart[a.order_rank[q]];
        ready_at = 0;
        began = progress_at = wall_clock64();
        waited = 0;
        idle_polls = 0;
        staged = false;
      } else {
        finished = true;
      }
    }
    if (ballot(pos >= 0) == 0) break;
    const uint64_t now = wall_clock64();
    bool go = false;
    uint64_t behind = 0;
    if (pos >= 0 && now >= ready_at) {
      uint64_t d = 0;
      if (t.tl == 0) d = ld_word(&a.ctl->ticket);  // transactions done so far
      d = (uint64_t)__shfl((long long)d, t.tb, 64);
      go = d >= need;
      behind = go ? 0 : need - d;
    }
    // Stage the operations (they do not change during the run).  A team whose
    // K-set cannot start yet does it now, so that the loads overlap its wait;
    // a team that can start does it on its way, after the gate's load, which
    // then never queues behind them.
    const bool stage = pos >= 0 && !staged;
    if (ballot(stage)) {
      if (stage) {
        const DevTxn d = a.txns[txn];
        first = d.first;
        n = d.n;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
        if (stage) {
          rowk[k] = 0;
          elem[k] = 0;
          arg[k] = 0;
          if (idx < n) {
            const DevOp op = a.ops[first + idx];
            rowk[k] = op.rowk;
            elem[k] = op.elem;
            arg[k] = op.arg;
          }
        }
      }
      staged = staged || stage;
    }
    bool done_now = false;
    if (ballot(go)) {
      if (STRICT) order_point<STRICT>();
      else asm volatile("" ::: "memory");
      int64_t x[K];
      bool v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
        v[k] = go && idx < n;
        x[k] = 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (v[k]) x[k] = ld_val(a.data + elem[k]);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (v[k]) st_val(a.reads + first + t.tl + k * L, x[k]);
      if (a.has_slot) order_point<STRICT>();  // slot writes read their sources back
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!v[k]) continue;
        const uint32_t kind = op_kind(rowk[k]);
        if (kind == CC_READ) continue;
        const int64_t src = kind == CC_WRITE_SLOT ? ld_val(a.reads + first + (uint32_t)(arg[k] & 0xFF)) : 0;
        st_val(a.data + elem[k], apply_op(kind, x[k], arg[k], src));
      }
      order_point<STRICT>();  // the K-set's writes are performed before it counts as done
      done_now = go;
    }
    (void)t.claim(&a.ctl->ticket, done_now, 1);
    if (pos >= 0) {
      const uint64_t after = wall_clock64();
      if (done_now) {
        if (t.tl == 0) {
          DevOutcome o;
          o.status = CC_COMMITTED;
          o.attempts = 1;
          o.serial_hi = a.order_rank[pos];
          o.serial_lo = txn;
          o.commit_ns = (int64_t)(((after - start_clock) * a.ns_per_tick_q16) >> 16);
          a.out[txn] = o;
          ++n_commit;
          t_wait += waited;
          t_useful += (after - began) - waited;
        }
        pos = -1;
      } else {
        waited += after - now;
        if (behind > 1) {
          const uint64_t cap = 4096ull * a.poll_ticks;
          const uint64_t nap = (behind - 1) * a.poll_ticks / 16;  // many transactions finish at once
          ready_at = after + (nap < cap ? nap : cap);
        }
        ++idle_polls;
        if (after - progress_at > a.wait_limit_ticks) {
          st_word(&a.ctl->stop, 1);
          finished = true;
          pos = -1;
        } else if ((idle_polls & 255u) == 255u && ld_word(&a.ctl->stop) != 0) {
          finished = true;
          pos = -1;
        }
      }
    }
    if (ballot(pos >= 0 && !done_now) && !ballot(go)) __builtin_amdgcn_s_sleep(2);
  }
  const uint64_t c0 = wave_sum(n_commit), c1 = wave_sum(t_useful), c2 = wave_sum(t_wait);
  if (t.lane == 0) {
    if (c0) {
      atomicAdd((unsigned long long *)&a.ctl->stats[DS_COMMITTED], (unsigned long long)c0);
      atomicAdd((unsigned long long *)&a.ctl->stats[DS_ATTEMPTS], (unsigned long long)c0);
      atomicMax((unsigned long long *)&a.ctl->stats[DS_MAX_ATTEMPTS], 1ull);
    }
    if (c1) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_USEFUL], (unsigned long long)c1);
    if (c2) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_WAIT], (unsigned long long)c2);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <int L, int K, bool STRICT>
static hipError_t gputx_launch_one(hipStream_t s, int waves_per_wg, int grid, const GputxArgs &a, int n_cu,
                                   bool exec, int *grid_used) {
  const int block = 64 * waves_per_wg;
  if (block > MaxThreads<K>::value) return hipErrorInvalidConfiguration;
  if (grid <= 0) grid = n_cu;  // one workgroup per compute unit, as GaccO
  const uint64_t teams_per_wg = (uint64_t)waves_per_wg * (64 / L);
  const uint64_t need = (a.n_txns + teams_per_wg - 1) / teams_per_wg;
  if ((uint64_t)grid > need) grid = (int)(need > 0 ? need : 1);
  *grid_used = grid;
  if (exec)
    hipLaunchKernelGGL((gputx_exec_kernel<L, K, STRICT>), dim3(grid), dim3(block), 0, s, a);
  else if (a.packed)
    hipLaunchKernelGGL((gputx_rank_kernel<L, K, STRICT, true>), dim3(grid), dim3(block), 0, s, a);
  else
    hipLaunchKernelGGL((gputx_rank_kernel<L, K, STRICT, false>), dim3(grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <bool STRICT>
static hipError_t gputx_dispatch(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid,
                                 const GputxArgs &a, int n_cu, bool exec, int *grid_used) {
  const int need_k = (max_ops + lanes - 1) / lanes;
#define CCE_TRY(LL, KK)             \
  if (lanes == LL && need_k <= KK) \
    return gputx_launch_one<LL, KK, STRICT>(s, waves_per_wg, grid, a, n_cu, exec, grid_used);
  CCE_TRY(1, 4)
  CCE_TRY(1, 16)
  CCE_TRY(4, 4)
  CCE_TRY(4, 16)
  CCE_TRY(16, 1)
  CCE_TRY(16, 4)
  CCE_TRY(64, 1)
  CCE_TRY(64, 4)
#undef CCE_TRY
  return hipErrorInvalidValue;
}

hipError_t launch_gputx_pass(hipStream_t s, bool exec, int lanes, int max_ops, int waves_per_wg, int grid,
                             bool strict, const GputxArgs &a, int n_cu, int *grid_used) {
  return strict ? gputx_dispatch<true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, exec, grid_used)
                : gputx_dispatch<false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, exec, grid_used);
}

hipError_t gputx_init_state(hipStream_t s, uint64_t *kstate, uint64_t n_rows, uint32_t *iota, uint64_t n_txns) {
  const uint64_t n = n_rows > n_txns ? n_rows : n_txns;
  const uint64_t blocks = (n + 255) / 256;
  if (blocks) hipLaunchKernelGGL(gputx_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, kstate, n_rows, iota,
                                 n_txns);
  return hipGetLastError();
}

hipError_t gputx_reset(hipStream_t s, Ctl *ctl) {
  hipLaunchKernelGGL(gputx_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

hipError_t gputx_kstart(hipStream_t s, const uint32_t *rank_sorted, uint64_t n, uint32_t *kstart) {
  const uint64_t blocks = (n + 255) / 256;
  if (blocks) hipLaunchKernelGGL(gputx_kstart_kernel, dim3((unsigned)blocks), dim3(256), 0, s, rank_sorted, n, kstart);
  return hipGetLastError();
}

}  // namespace cce
