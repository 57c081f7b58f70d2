// GaccO execution kernel: persistent teams hand every row to its accessors in
// transaction-id order, using the lock table built by the preprocessing
// (gacco.hip).  No transaction aborts; each runs once.
#include "opset.h"
#include "txn_kernel.h"

namespace cce {

template <int L, int K, bool STRICT>
__global__ void __launch_bounds__(MaxThreads<K>::value) gacco_kernel(GaccoArgs a) {
  constexpr int NW = L == 64 ? K : 1;
  static_assert(L == 64 || L * K <= 64, "operation sets of one word");
  using Set = OpSet<NW>;
  Team<L> t;
  const uint64_t start_clock = a.ctl->start_clock;
  int64_t txn = -1;  // team-uniform
  bool finished = false;
  uint32_t first = 0;
  uint32_t rowk[K], elem[K], rk[K];
  int64_t arg[K], x[K];
  Set valid = Set::zero(), lead = Set::zero(), fol = Set::zero(), slot = Set::zero();
  Set granted = Set::zero(), done = Set::zero(), released = Set::zero();
  uint64_t ready_at = 0, began = 0, progress_at = 0, waited = 0;
  uint32_t idle_polls = 0;
  uint64_t n_commit = 0, t_useful = 0, t_wait = 0;

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
    uint64_t now = wall_clock64();
    if (ballot(fresh)) {
      // stage the transaction's operations (coalesced 16 B loads per team)
      uint32_t n = 0;
      if (fresh) {
        const DevTxn d = a.txns[txn];
        first = d.first;
        n = d.n;
      }
      bool v[K], ld[K], fo[K], sl[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
        v[k] = fresh && idx < n;
        ld[k] = fo[k] = sl[k] = false;
        if (v[k]) {
          const DevOp op = a.ops[first + idx];
          rowk[k] = op.rowk;
          elem[k] = op.elem;
          arg[k] = op.arg;
          ld[k] = op_leader(op.rowk);
          fo[k] = !ld[k];
          sl[k] = op_kind(op.rowk) == CC_WRITE_SLOT;
          rk[k] = ld[k] ? a.rank[first + idx] : 0u;
        }
      }
      const Set sv = team_set<L, K, NW>(t, v), sld = team_set<L, K, NW>(t, ld), sfo = team_set<L, K, NW>(t, fo),
                ssl = team_set<L, K, NW>(t, sl);
      if (fresh) {
        valid = sv;
        lead = sld;
        fol = sfo;
        slot = ssl;
        granted = done = released = Set::zero();
        ready_at = 0;
        began = progress_at = now;
        waited = 0;
        idle_polls = 0;
      }
    }
    const bool act = txn >= 0 && now >= ready_at;

    // 1. look at the words of the rows this team still waits for
    bool g[K];
    uint64_t ahead = ~0ull;  // fewest accesses queued before one of my waiting rows
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t i = (uint32_t)t.tl + (uint32_t)(k * L);
      g[k] = false;
      if (act && lead.test(i) && !granted.test(i)) {
        const uint64_t w = ld_word(a.words + op_row(rowk[k]));
        // turn mode: the word is the position whose turn it is; shared
        // reads: a write needs every earlier access done, a read every
        // earlier write
        const uint64_t have = !a.shared ? w : (op_written(rowk[k]) ? (w >> 32) : (w & 0xFFFFFFFFull));
        g[k] = a.shared ? have >= (uint64_t)rk[k] : have == (uint64_t)rk[k];
        if (!g[k] && (uint64_t)rk[k] > have) {
          const uint64_t d = (uint64_t)rk[k] - have;
          ahead = d < ahead ? d : ahead;
        }
      }
    }
    const Set newly = team_set<L, K, NW>(t, g);
    if (act) granted = granted | newly;

    // 2. run the operations whose row has come to the transaction (a slot
    //    write also needs its source operation done)
    const Set runnable = spread_up(granted, fol) & valid & ~done;
    bool r[K];
    bool any_r = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t i = (uint32_t)t.tl + (uint32_t)(k * L);
      r[k] = act && runnable.test(i);
      if (r[k] && slot.test(i)) r[k] = done.test((uint32_t)(arg[k] & 0xFF));
      any_r |= r[k];
    }
    if (ballot(any_r)) {
      // Each operation is one memory round trip: the row is this
      // transaction's alone until it is passed on, so a read is a load, an
      // add is a fetch-add (returning the pre-image), a slot write an
      // exchange.  The turn was seen before any of them is issued (they
      // depend on it); a slot write first waits for its source's read value,
      // stored in an earlier step.
      bool any_slot = false;
#pragma unroll
      for (int k = 0; k < K; ++k) any_slot |= r[k] && slot.test((uint32_t)t.tl + (uint32_t)(k * L));
      if (STRICT || ballot(any_slot)) order_point<STRICT>();
      else asm volatile("" ::: "memory");
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!r[k]) continue;
        const uint32_t kind = op_kind(rowk[k]);
        uint64_t *cell = (uint64_t *)(a.data + elem[k]);
        if (kind == CC_READ) {
          x[k] = ld_val(a.data + elem[k]);
        } else if (kind == CC_ADD || kind == CC_COND_ADD) {
          x[k] = (int64_t)add_word(cell, (uint64_t)arg[k]);
        } else {
          const int64_t src = ld_val(a.reads + first + (uint32_t)(arg[k] & 0xFF));
          x[k] = (int64_t)xchg_word(cell, (uint64_t)apply_op(CC_WRITE_SLOT, 0, arg[k], src));
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        // the replenishing rule of a conditional add, applied while the row is still held
        if (r[k] && op_kind(rowk[k]) == CC_COND_ADD &&
            (int64_t)((uint64_t)x[k] + (uint64_t)arg[k]) < CC_COND_LO)
          add_word((uint64_t *)(a.data + elem[k]), (uint64_t)CC_COND_HI);
      }
    }
    const Set ran = team_set<L, K, NW>(t, r);
    if (act) done = done | ran;

    // 3. pass on every row whose whole group has run
    const Set rel = lead & granted & ~released & ~gather_down(valid & ~done, fol);
    bool rl[K];
    bool any_rl = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t i = (uint32_t)t.tl + (uint32_t)(k * L);
      rl[k] = act && rel.test(i);
      any_rl |= rl[k];
    }
    if (ballot(any_rl)) {
      order_point<STRICT>();  // the group's updates are performed before the row moves on
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!rl[k]) continue;
        if (a.shared) add_word(a.words + op_row(rowk[k]), (1ull << 32) | (op_written(rowk[k]) ? 1ull : 0ull));
        else st_word(a.words + op_row(rowk[k]), (uint64_t)rk[k] + 1);
      }
    }
    // read values leave after the releases, so that no release waits for them
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (r[k]) __builtin_nontemporal_store(x[k], a.reads + first + t.tl + k * L);
    if (act) released = released | rel;

    // 4. bookkeeping: completion, sleep in proportion to the queue ahead,
    //    and the bounded wait
    if (txn >= 0) {
      const uint64_t after = wall_clock64();
      const bool progressed = act && !((ran == Set::zero()) && (newly == Set::zero()));
      if (act && done == valid && (released == (lead & valid))) {
        if (t.tl == 0) {
          DevOutcome o;
          o.status = CC_COMMITTED;
          o.attempts = 1;
          o.serial_hi = 0;
          o.serial_lo = (uint64_t)txn;
          o.commit_ns = (int64_t)(((after - start_clock) * a.ns_per_tick_q16) >> 16);
          a.out[txn] = o;
          ++n_commit;
          t_wait += waited;
          t_useful += (after - began) - waited;
        }
        txn = -1;
      } else if (progressed) {
        progress_at = after;
        idle_polls = 0;
      } else {
        const uint64_t d = t.max(~ahead);  // team minimum of `ahead`
        const uint64_t m = ~d;
        if (act) {
          if (m != ~0ull && m > 1) {
            const uint64_t cap = 4096ull * a.poll_ticks;  // look again within ~1 ms at most
            const uint64_t nap = (m - 1) * a.poll_ticks;
            ready_at = after + (nap < cap ? nap : cap);
          }
          ++idle_polls;
        }
        waited += after - now;
        if (after - progress_at > a.wait_limit_ticks) {
          // cannot happen while the lock table is consistent; stop every team
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

template <int L, int K, bool STRICT>
static hipError_t gacco_launch_one(hipStream_t s, int waves_per_wg, int grid, const GaccoArgs &a, int n_cu,
                                   int *grid_used) {
  auto kern = gacco_kernel<L, K, STRICT>;
  const int block = 64 * waves_per_wg;
  if (block > MaxThreads<K>::value) return hipErrorInvalidConfiguration;
  if (grid <= 0) {
    // default: one workgroup per compute unit.  Measured on the key-value
    // workload (1M transactions x 16 ops): at Zipf 0.9 and 0.99 the run is
    // twice as fast as with every workgroup that fits at once, because the
    // teams queued on a hot row slow its hand-offs with their looks at its
    // word; at Zipf 0 and 0.6 the difference is within 20%.
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    grid = n_cu;
  }
  const uint64_t teams_per_wg = (uint64_t)waves_per_wg * (64 / L);
  const uint64_t need = (a.n_txns + teams_per_wg - 1) / teams_per_wg;
  if ((uint64_t)grid > need) grid = (int)(need > 0 ? need : 1);
  *grid_used = grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <bool STRICT>
static hipError_t gacco_dispatch(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid,
                                 const GaccoArgs &a, int n_cu, int *grid_used) {
  const int need_k = (max_ops + lanes - 1) / lanes;
#define CCE_TRY(LL, KK)             \
  if (lanes == LL && need_k <= KK) \
    return gacco_launch_one<LL, KK, STRICT>(s, waves_per_wg, grid, a, n_cu, grid_used);
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

hipError_t launch_gacco(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, bool strict,
                        const GaccoArgs &a, int n_cu, int *grid_used) {
  return strict ? gacco_dispatch<true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                : gacco_dispatch<false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
}

}  // namespace cce
