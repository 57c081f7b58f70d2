// The plain-batch transaction kernel, templated on lanes per transaction,
// register slots per lane, scheme and fence strength, and its launcher.
// Each scheme instantiates it in its own translation unit (txn_<scheme>.hip).
#pragma once

#include "schemes.h"

namespace cce {

template <int L, int K, int SCHEME, bool STRICT, bool LATCH>
__device__ __forceinline__ int attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a, uint32_t txn,
                                       bool retry, bool resume, bool may_wait, uint64_t *hi, uint64_t *lo) {
  const bool precheck = a.precheck == 2 || (a.precheck == 1 && retry);
  if constexpr (SCHEME == CC_OCC) return occ_attempt<L, K, STRICT, LATCH>(t, s, active, a, precheck, hi, lo);
  else if constexpr (SCHEME == CC_2PL_NW) return tpl_attempt<L, K, STRICT, LATCH>(t, s, active, a, txn, hi, lo);
  else if constexpr (SCHEME == CC_2PL_WD)
    return tplwd_attempt<L, K, STRICT, LATCH>(t, s, active, a, txn, resume, may_wait, hi, lo);
  else if constexpr (SCHEME == CC_TO) return to_attempt<L, K, STRICT, false, LATCH>(t, s, active, a, precheck, hi, lo);
  else if constexpr (SCHEME == CC_MVCC) return to_attempt<L, K, STRICT, true, LATCH>(t, s, active, a, precheck, hi, lo);
  else return tictoc_attempt<L, K, STRICT, LATCH>(t, s, active, a, precheck, hi, lo);
}

// ---------------------------------------------------------------------------
// Plain batch kernel: persistent teams, in-kernel retry until commit (or
// deferral to the next, less concurrent pass).
// ---------------------------------------------------------------------------
template <int L, int K, int SCHEME, bool STRICT, bool LATCH>
__global__ void __launch_bounds__(MaxThreads<K>::value) txn_kernel(RunArgs a) {
  Team<L> t;
  Slots<K> s;
  const uint64_t start_clock = a.ctl->start_clock;
  // epoch mode replays a captured graph, so the pending count is read here
  const uint64_t n_txns = a.n_from_ctl ? ld_word(&a.ctl->pending_n) : a.n_txns;
  int64_t txn = -1;         // current transaction (team-uniform)
  uint32_t attempts = 0;    // attempts of txn so far, all passes
  uint32_t pass_att = 0;    // attempts of txn in this pass
  uint64_t ready_at = 0;    // wall-clock tick before which the team waits
  bool done = false;        // no transactions left for this team
  uint64_t n_commit = 0, n_att = 0, n_lock = 0, n_valid = 0, n_gave = 0, n_defer = 0, n_ovf = 0, max_att = 0;
  uint64_t t_useful = 0, t_abort = 0, t_wait = 0;  // per team, in leader lanes
  uint64_t reserved = 0;    // serving: bytes this team's transaction reserved (0: none)
  uint64_t res_pos = 0;     // serving: the reservation's position in the byte queue
  bool admitted = false;    // serving: the reservation has been granted
  uint64_t t_round[4] = {0, 0, 0, 0};  // OCC committed attempts: per-round ticks
  uint64_t n_admit_wait = 0;
  bool resume = false;      // 2PL wait-die: the team waits holding locks; its next attempt continues this one
  uint32_t waits = 0;       // 2PL wait-die: waits of the current attempt
  uint64_t n_waits = 0;
  uint64_t n_hot_acq = 0, n_hot_fail = 0, t_hot = 0;  // OCC: the most written row, in the lane holding it
  uint32_t wait_row = ~0u;  // CC_RUN_WAIT_BLOCKER: the held row the team waits for (~0u: not waiting)
  uint64_t wait_since = 0, next_poll = 0;
  uint64_t n_blocked = 0;   // waits entered

  for (;;) {
    if constexpr (LATCH) {
      // a stuck latch failed the run (see latched): every team leaves its
      // transaction pending and exits
      if (__shfl((int)(ld_word(&a.ctl->stop) != 0), 0, 64)) break;
    }
    const bool need = txn < 0 && !done;
    const uint64_t q = t.claim(&a.ctl->queue, need, 1);
    if (need) {
      if (q < n_txns) {
        txn = a.list ? (int64_t)a.list[q] : (int64_t)q;
        attempts = a.pass ? a.out[txn].attempts : 0;
        pass_att = 0;
        // serving: not before the transaction's arrival
        ready_at = a.arrival ? start_clock + (uint64_t)a.arrival[txn] : 0;
        reserved = 0;
        admitted = false;
        resume = false;
        waits = 0;
        wait_row = ~0u;
      } else {
        done = true;
      }
    }
    if (ballot(txn >= 0) == 0) break;
    uint64_t now = wall_clock64();
    if (a.budget_cap && txn >= 0 && now >= ready_at && !admitted) {
      // serving admission, first come first served on bytes: an arrived
      // transaction takes a position in a byte queue with one fetch_add on
      // the reserved counter, and runs once the released counter shows that
      // all but `cap` of the bytes queued before it (and its own) have been
      // given back.  Waiting is a load; nothing is undone, so concurrent
      // admissions cannot crowd each other out.  A transaction larger than
      // the cap waits for everything before it, then runs alone.
      uint64_t rs = reserved, pos = res_pos;
      bool ok = false;
      if (t.tl == 0) {
        if (rs == 0) {
          rs = (uint64_t)a.txns[txn].n * a.bytes_per_op + 1;
          pos = add_word(&a.ctl->budget_reserved, rs);
        }
        const uint64_t need = rs < a.budget_cap ? rs : a.budget_cap;
        ok = ld_word(&a.ctl->budget_released) + a.budget_cap >= pos + need;
        if (!ok) ++n_admit_wait;
      }
      reserved = (uint64_t)__shfl((long long)rs, t.tb, 64);
      res_pos = (uint64_t)__shfl((long long)pos, t.tb, 64);
      admitted = __shfl((int)ok, t.tb, 64) != 0;
      if (!admitted) ready_at = now + 1 + (mix64(((uint64_t)txn << 20) ^ now) % (4ull * a.backoff_ticks));
    }
    if (a.wait_blocker) {
      // a waiting team looks at its row's word, at randomised intervals, until
      // the row is free or the wait times out; then it retries after a jitter.
      // Every wait ends: the time-out bounds it, and the final pass, which
      // never defers, never waits (the team loop's CPU model checks this rule).
      const bool poll = txn >= 0 && wait_row != ~0u && now >= next_poll;  // team-uniform
      bool free_now = false;
      if (poll && t.tl == 0)
        free_now = !(ld_word(a.words + wait_row) & (1ull << 63)) || now - wait_since > a.wait_max_ticks;
      free_now = __shfl((int)free_now, t.tb, 64) != 0;
      if (poll) {
        const uint64_t r = mix64(((uint64_t)txn << 24) ^ now);
        if (free_now) {
          wait_row = ~0u;
          ready_at = now + r % ((uint64_t)a.jitter_ticks + 1);
        } else {
          next_poll = now + a.poll_ticks / 2 + r % ((uint64_t)a.poll_ticks + 1);
        }
      }
    }
    const bool active = txn >= 0 && now >= ready_at;
    if (ballot(active) == 0) {
      __builtin_amdgcn_s_sleep(2);
      if (txn >= 0 && t.tl == 0) t_wait += wall_clock64() - now;
      continue;
    }
    // stage the transaction's ops in registers (coalesced 16 B loads per team)
    uint32_t first = 0, n = 0;
    if (active) {
      const DevTxn d = a.txns[txn];
      first = d.first;
      n = d.n;
    }
    // a waiting team (2PL wait-die) keeps its staged operations and locks
    const bool keep = SCHEME == CC_2PL_WD && resume;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (keep) continue;
      const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
      s.valid[k] = active && idx < n;
      s.oi[k] = first + idx;
      if (s.valid[k]) {
        const DevOp op = a.ops[first + idx];
        s.rowk[k] = op.rowk;
        s.elem[k] = op.elem;
        s.arg[k] = op.arg;
      } else {
        s.rowk[k] = FOLLOWER_BIT;
        s.elem[k] = 0;
        s.arg[k] = 0;
      }
      s.x[k] = 0;
      s.v[k] = 0;
    }
    uint64_t key_hi = 0, key_lo = 0;
    s.block = ~0u;
    const int r = attempt<L, K, SCHEME, STRICT, LATCH>(t, s, active, a, (uint32_t)(txn < 0 ? 0 : txn), attempts >= 1,
                                                keep, waits < a.wd_wait_limit, &key_hi, &key_lo);
    if (t.tl == 0 && txn >= 0) {
      const uint64_t dt = wall_clock64() - now;
      if (!active || r == WAITING) t_wait += dt;
      else if (r == COMMIT) t_useful += dt;
      else t_abort += dt;
      if constexpr (SCHEME == CC_OCC) {
        if (active && r == COMMIT) {
          t_round[0] += s.tr[0] - now;
          t_round[1] += s.tr[1] - s.tr[0];
          t_round[2] += s.tr[2] - s.tr[1];
          t_round[3] += s.tr[3] - s.tr[2];
        }
      }
    }
    if constexpr (SCHEME == CC_OCC) {
      if (active && s.hot_got) {
        ++n_hot_acq;
        n_hot_fail += r != COMMIT;
        t_hot += s.hot_dt;
      }
    }
    if (active && r == WAITING) {
      // wait-die: keep the locks and try the missing ones again shortly (a
      // wait is not an attempt; an attempt's waits are bounded)
      ++waits;
      if (t.tl == 0) ++n_waits;
      resume = true;
      ready_at = now + 1 + (mix64(((uint64_t)txn << 20) ^ waits) % ((uint64_t)a.backoff_ticks * (1 + (waits < 8 ? waits : 8))));
    } else if (active) {
      resume = false;
      waits = 0;
      ++attempts;
      ++pass_att;
      ++n_att;
      if (r == COMMIT) {
        if (t.tl == 0) {
          DevOutcome o;
          o.status = CC_COMMITTED;
          o.attempts = attempts;
          o.serial_hi = key_hi;
          o.serial_lo = key_lo;
          const uint64_t dt = wall_clock64() - start_clock;
          o.commit_ns = (int64_t)((dt * a.ns_per_tick_q16) >> 16);
          a.out[txn] = o;
          ++n_commit;
          max_att = attempts > max_att ? attempts : max_att;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (s.valid[k]) __builtin_nontemporal_store(s.x[k], a.reads + first + t.tl + k * L);
        if (reserved && t.tl == 0) add_word(&a.ctl->budget_released, reserved);
        reserved = 0;
        txn = -1;
      } else {
        if (t.tl == 0) {
          if (r == ABORT_LOCK) ++n_lock;
          else if (r == ABORT_VALID) ++n_valid;
          else ++n_ovf;
        }
        if (r == TS_OVERFLOW || attempts >= a.max_attempts || (a.defer_after && pass_att >= a.defer_after)) {
          // give up (timestamp overflow, attempt limit) or leave the
          // transaction to the next, less concurrent pass
          if (t.tl == 0) {
            a.out[txn].attempts = attempts;
            if (r == TS_OVERFLOW || attempts >= a.max_attempts) ++n_gave; else ++n_defer;
            max_att = attempts > max_att ? attempts : max_att;
            if (reserved) add_word(&a.ctl->budget_released, reserved);
          }
          reserved = 0;
          txn = -1;
        } else if (a.wait_blocker && a.defer_after && s.block != ~0u) {
          // wait for the row another transaction held (passes that defer only)
          wait_row = s.block;
          wait_since = now;
          next_poll = now + a.poll_ticks;
          ready_at = ~0ull;
          if (t.tl == 0) ++n_blocked;
        } else {
          // randomised exponential back-off
          const uint32_t sh = pass_att < 12 ? pass_att : 12;
          const uint64_t span = (uint64_t)a.backoff_ticks << sh;
          ready_at = now + (mix64(((uint64_t)txn << 20) ^ attempts) % (span + 1));
        }
      }
    }
  }
  // one atomic per counter per wavefront (team leaders hold the counts)
  n_att = t.tl == 0 ? n_att : 0;
  const uint64_t c0 = wave_sum(n_commit), c1 = wave_sum(n_att), c2 = wave_sum(n_lock), c3 = wave_sum(n_valid),
                 c4 = wave_sum(n_gave), c5 = wave_max(max_att), c6 = wave_sum(n_defer), c7 = wave_sum(n_ovf);
  const uint64_t c8 = wave_sum(t_useful), c9 = wave_sum(t_abort), c10 = wave_sum(t_wait),
                 c11 = wave_sum(n_admit_wait), c13 = wave_sum(n_waits);
  const uint64_t c14 = wave_sum(n_hot_acq), c15 = wave_sum(n_hot_fail), c16 = wave_sum(t_hot),
                 c17 = wave_sum(n_blocked);
  uint64_t cr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cr[i] = wave_sum(t_round[i]);
  if (t.lane == 0) {
    if (c0) atomicAdd((unsigned long long *)&a.ctl->stats[DS_COMMITTED], (unsigned long long)c0);
    if (c1) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ATTEMPTS], (unsigned long long)c1);
    if (c2) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_LOCK], (unsigned long long)c2);
    if (c3) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_VALID], (unsigned long long)c3);
    if (c4) atomicAdd((unsigned long long *)&a.ctl->stats[DS_GAVE_UP], (unsigned long long)c4);
    if (c5) atomicMax((unsigned long long *)&a.ctl->stats[DS_MAX_ATTEMPTS], (unsigned long long)c5);
    if (c6) atomicAdd((unsigned long long *)&a.ctl->stats[DS_DEFERRED], (unsigned long long)c6);
    if (c7) atomicAdd((unsigned long long *)&a.ctl->stats[DS_TS_OVERFLOW], (unsigned long long)c7);
    if (c8) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_USEFUL], (unsigned long long)c8);
    if (c9) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_ABORT], (unsigned long long)c9);
    if (c10) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_WAIT], (unsigned long long)c10);
    if (c11) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ADMIT_WAITS], (unsigned long long)c11);
    if (c13) atomicAdd((unsigned long long *)&a.ctl->stats[DS_WD_WAITS], (unsigned long long)c13);
    if (c14) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_ACQ], (unsigned long long)c14);
    if (c15) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_FAILED], (unsigned long long)c15);
    if (c16) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_HOLD], (unsigned long long)c16);
    if (c17) atomicAdd((unsigned long long *)&a.ctl->stats[DS_BLOCKED_WAITS], (unsigned long long)c17);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (cr[i]) atomicAdd((unsigned long long *)&a.ctl->stats[DS_R1 + i], (unsigned long long)cr[i]);
  }
}

// ---------------------------------------------------------------------------
// dispatch over (lanes per txn, ops per lane, strict, latch)
// ---------------------------------------------------------------------------
template <int L, int K, int SCHEME, bool STRICT, bool LATCH>
static hipError_t launch_one(hipStream_t s, int waves_per_wg, int grid, const RunArgs &a, int n_cu, int *grid_used) {
  auto kern = txn_kernel<L, K, SCHEME, STRICT, LATCH>;
  const int block = 64 * waves_per_wg;
  if (block > MaxThreads<K>::value) return hipErrorInvalidConfiguration;
  if (grid <= 0) {
    // default: one workgroup per compute unit.  Measured on the key-value
    // workload, fuller occupancy only adds conflicting transactions in flight
    // (more aborts) without adding throughput, at every contention level.
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    grid = n_cu;
  }
  // never more teams than transactions
  const uint64_t teams_per_wg = (uint64_t)waves_per_wg * (64 / L);
  const uint64_t need = (a.n_txns + teams_per_wg - 1) / teams_per_wg;
  if ((uint64_t)grid > need) grid = (int)(need > 0 ? need : 1);
  *grid_used = grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int SCHEME, bool STRICT, bool LATCH>
static hipError_t dispatch(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, const RunArgs &a,
                           int n_cu, int *grid_used) {
  const int need_k = (max_ops + lanes - 1) / lanes;
#define CCE_TRY(LL, KK)                                                                      \
  if (lanes == LL && need_k <= KK)                                                           \
    return launch_one<LL, KK, SCHEME, STRICT, LATCH>(s, waves_per_wg, grid, a, n_cu, grid_used);
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

}  // namespace cce
