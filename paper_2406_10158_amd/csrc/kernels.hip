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
#include "engine.h"

namespace cce {

constexpr uint64_t LOCK = 1ull << 63;

// ---------------------------------------------------------------------------
// memory helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ld_word(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t or_word(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_val(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_val(int64_t *p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool STRICT>
__device__ __forceinline__ void order_point() {
  if constexpr (STRICT) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  } else {
    // compiler barrier for the atomics around it, then wait until every
    // memory operation this wavefront issued has completed
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
  }
}

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

template <int L>
struct Team {
  int lane, tl, tb;  // lane in wave, lane in team, team base lane
  uint64_t tmask;    // this team's lanes
  __device__ __forceinline__ Team() {
    lane = __lane_id();
    tl = lane & (L - 1);
    tb = lane - tl;
    tmask = (L == 64 ? ~0ull : ((1ull << L) - 1ull)) << tb;
  }
  // any lane of my team has p
  __device__ __forceinline__ bool any(bool p) const { return (ballot(p) & tmask) != 0; }
  // team leaders that ask (want, uniform per team) share one atomic add of
  // `per` per team on *ctr; returns the value before this team's share.
  __device__ __forceinline__ uint64_t claim(uint64_t *ctr, bool want, uint64_t per) const {
    uint64_t m = ballot(want && tl == 0);
    if (m == 0) return 0;
    int first = __ffsll((unsigned long long)m) - 1;
    uint64_t base = 0;
    if (lane == first)
      base = __hip_atomic_fetch_add(ctr, (uint64_t)__popcll(m) * per, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = readlane64(base, first);
    uint64_t below = m & ((1ull << tb) - 1ull);
    return base + (uint64_t)__popcll(below) * per;
  }
  // value of v in lane (tb + src_lane)
  __device__ __forceinline__ int64_t shfl(int64_t v, int src_lane) const { return __shfl(v, tb + src_lane, 64); }
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_max(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint64_t w = (uint64_t)__shfl_xor((long long)v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// new value of one operation from its pre-image (slot values already resolved)
__device__ __forceinline__ int64_t apply_op(uint32_t kind, int64_t pre, int64_t arg, int64_t slot_src) {
  switch (kind) {
    case CC_ADD:
      return (int64_t)((uint64_t)pre + (uint64_t)arg);
    case CC_COND_ADD: {
      int64_t v = (int64_t)((uint64_t)pre + (uint64_t)arg);
      return v < CC_COND_LO ? (int64_t)((uint64_t)v + (uint64_t)CC_COND_HI) : v;
    }
    case CC_WRITE_SLOT: {
      uint64_t a = (uint64_t)arg;
      int64_t mul = (int64_t)((a >> 8) & 0xFFFFFFull);
      mul = (mul ^ 0x800000) - 0x800000;  // sign-extend 24 bits
      int64_t add = (int64_t)(int32_t)(uint32_t)(a >> 32);
      return (int64_t)((uint64_t)slot_src * (uint64_t)mul + (uint64_t)add);
    }
    default:
      return pre;
  }
}

// Per-lane operation slots of the current transaction.
template <int K>
struct Slots {
  uint32_t rowk[K];
  uint32_t elem[K];
  int64_t arg[K];
  uint64_t v[K];   // control word observed / held
  int64_t x[K];    // pre-image read
  bool got[K];     // this slot's row lock is held
  bool valid[K];
};

__device__ __forceinline__ uint32_t op_row(uint32_t rk) { return rk & ROW_MASK; }
__device__ __forceinline__ uint32_t op_kind(uint32_t rk) { return (rk >> KIND_SHIFT) & 3u; }
__device__ __forceinline__ bool op_leader(uint32_t rk) { return !(rk & FOLLOWER_BIT); }
__device__ __forceinline__ bool op_written(uint32_t rk) { return (rk & WRITTEN_BIT) != 0; }

// Value read by op `src` of the team's transaction (lane src%L, slot src/L).
template <int L, int K>
__device__ __forceinline__ int64_t slot_source(const Team<L> &t, const Slots<K> &s, uint32_t src) {
  int64_t r = 0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    int64_t y = t.shfl(s.x[kk], (int)(src & (L - 1)));
    if ((int)(src / L) == kk) r = y;
  }
  return r;
}

enum AttemptResult { COMMIT = 0, ABORT_LOCK = 1, ABORT_VALID = 2 };

// ---------------------------------------------------------------------------
// OCC (Silo-style; paper Section 2 "Optimistic Concurrency Control" and
// Section 3.5 "OCC", control word = lock bit + 63-bit TID, Table 2).
//
// One attempt, in four wavefront-synchronous rounds:
//   R1  write-set rows: try-lock by fetch_or(LOCK) -- the returned word is the
//       row's committed TID; a set lock bit means another transaction holds
//       it and we abort (no-wait, as in the paper's Silo and TicToc).
//       read-set rows: load the TID word; locked -> abort.
//   R2  read every operation's value (write rows under our lock); draw the
//       serial ticket, which also becomes the TID of rows we install.
//   R3  validate: each read-only row's word is unchanged and its TID is
//       older than our ticket; abort otherwise (releasing our locks).
//   R4  store new values, wait, then store each write row's word = ticket,
//       which publishes the values and releases the lock in one store.
// The paper's Silo locks its write set at validation time, after the read
// phase; here read/write sets are known in advance (Section 4.1
// "Constraints"), so write rows are locked first and read under the lock,
// which shortens the window during which a hot row is held or can be
// invalidated.  Serial order = ticket order (proof in the design doc terms):
// tickets are drawn while all write locks are held and before validation.
// ---------------------------------------------------------------------------
template <int L, int K, bool STRICT>
__device__ __forceinline__ int occ_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                           uint64_t *ticket_out) {
  bool fail = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    if (active && s.valid[k] && op_leader(s.rowk[k])) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      if (op_written(s.rowk[k])) {
        uint64_t old = or_word(w, LOCK);
        s.v[k] = old;
        s.got[k] = !(old & LOCK);
        fail |= !s.got[k];
      } else {
        uint64_t o = ld_word(w);
        s.v[k] = o;
        fail |= (o & LOCK) != 0;
      }
    }
  }
  order_point<STRICT>();
  const bool lock_fail = t.any(fail);
  bool alive = active && !lock_fail;
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) st_word(a.words + op_row(s.rowk[k]), s.v[k]);
  }
  // R2: values and ticket
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.valid[k]) s.x[k] = ld_val(a.data + s.elem[k]);
  const uint64_t ticket = t.claim(&a.ctl->ticket, alive, 1) + 1;
  order_point<STRICT>();
  // R3: validation
  bool bad = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (alive && s.valid[k] && op_leader(s.rowk[k])) {
      if (!op_written(s.rowk[k])) bad |= ld_word(a.words + op_row(s.rowk[k])) != s.v[k];
      bad |= (s.v[k] & ~LOCK) >= ticket;
    }
  }
  const bool valid_fail = t.any(bad);
  const bool commit = alive && !valid_fail;
  if (alive && valid_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) st_word(a.words + op_row(s.rowk[k]), s.v[k]);
  }
  // R4: install and release
  if (a.has_slot) {
    int64_t src_val[K];
#pragma unroll
    for (int k = 0; k < K; ++k) src_val[k] = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint32_t src = (s.valid[k] && op_kind(s.rowk[k]) == CC_WRITE_SLOT) ? (uint32_t)(s.arg[k] & 0xFF) : 0u;
      src_val[k] = slot_source<L, K>(t, s, src);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ)
        st_val(a.data + s.elem[k], apply_op(op_kind(s.rowk[k]), s.x[k], s.arg[k], src_val[k]));
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ)
        st_val(a.data + s.elem[k], apply_op(op_kind(s.rowk[k]), s.x[k], s.arg[k], 0));
  }
  order_point<STRICT>();
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (commit && s.got[k]) st_word(a.words + op_row(s.rowk[k]), ticket);
  *ticket_out = ticket;
  if (!active) return COMMIT;
  return lock_fail ? ABORT_LOCK : (valid_fail ? ABORT_VALID : COMMIT);
}

// ---------------------------------------------------------------------------
// Plain batch kernel: persistent teams, in-kernel retry until commit.
// ---------------------------------------------------------------------------
// Largest workgroup a (lanes, ops-per-lane) variant is compiled for: more
// register slots per lane leave room for fewer wavefronts.
template <int K>
struct MaxThreads {
  static constexpr int value = K <= 1 ? 1024 : (K <= 4 ? 512 : 256);
};

template <int L, int K, int SCHEME, bool STRICT>
__global__ void __launch_bounds__(MaxThreads<K>::value) txn_kernel(RunArgs a) {
  Team<L> t;
  Slots<K> s;
  const uint64_t start_clock = a.ctl->start_clock;
  int64_t txn = -1;         // current transaction (team-uniform)
  uint32_t attempts = 0;    // attempts of txn so far, all passes
  uint32_t pass_att = 0;    // attempts of txn in this pass
  uint64_t ready_at = 0;    // wall-clock tick before which the team waits
  bool done = false;        // no transactions left for this team
  uint64_t n_commit = 0, n_att = 0, n_lock = 0, n_valid = 0, n_gave = 0, n_defer = 0, max_att = 0;

  for (;;) {
    const bool need = txn < 0 && !done;
    const uint64_t q = t.claim(&a.ctl->queue, need, 1);
    if (need) {
      if (q < a.n_txns) {
        txn = a.list ? (int64_t)a.list[q] : (int64_t)q;
        attempts = a.pass ? a.out[txn].attempts : 0;
        pass_att = 0;
        ready_at = 0;
      } else {
        done = true;
      }
    }
    if (ballot(txn >= 0) == 0) break;
    const uint64_t now = wall_clock64();
    const bool active = txn >= 0 && now >= ready_at;
    if (ballot(active) == 0) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    // stage the transaction's ops in registers (coalesced 16 B loads per team)
    uint32_t first = 0, n = 0;
    if (active) {
      const DevTxn d = a.txns[txn];
      first = d.first;
      n = d.n;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
      s.valid[k] = active && idx < n;
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
    uint64_t key = 0;
    int r = occ_attempt<L, K, STRICT>(t, s, active, a, &key);
    if (active) {
      ++attempts;
      ++pass_att;
      ++n_att;
      if (r == COMMIT) {
        if (t.tl == 0) {
          DevOutcome o;
          o.status = CC_COMMITTED;
          o.attempts = attempts;
          o.serial_hi = 0;
          o.serial_lo = key;
          const uint64_t dt = wall_clock64() - start_clock;
          o.commit_ns = (int64_t)((dt * a.ns_per_tick_q16) >> 16);
          a.out[txn] = o;
          ++n_commit;
          max_att = attempts > max_att ? attempts : max_att;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (s.valid[k]) __builtin_nontemporal_store(s.x[k], a.reads + first + t.tl + k * L);
        txn = -1;
      } else {
        if (t.tl == 0) {
          if (r == ABORT_LOCK) ++n_lock; else ++n_valid;
        }
        if (attempts >= a.max_attempts || (a.defer_after && pass_att >= a.defer_after)) {
          // give up (attempt limit) or leave it to the next, less concurrent pass
          if (t.tl == 0) {
            a.out[txn].attempts = attempts;
            if (attempts >= a.max_attempts) ++n_gave; else ++n_defer;
            max_att = attempts > max_att ? attempts : max_att;
          }
          txn = -1;
        } else {
          // randomised exponential back-off
          const uint32_t sh = pass_att < 12 ? pass_att : 12;
          const uint64_t span = (uint64_t)a.backoff_ticks << sh;
          ready_at = now + (mix64(((uint64_t)txn << 20) ^ attempts) % (span + 1));
        }
      }
    }
  }
  // one atomic per counter per wavefront (team leaders hold the counts; the
  // attempts counter is kept per lane and counted in leaders only)
  n_att = t.tl == 0 ? n_att : 0;
  const uint64_t c0 = wave_sum(n_commit), c1 = wave_sum(n_att), c2 = wave_sum(n_lock), c3 = wave_sum(n_valid),
                 c4 = wave_sum(n_gave), c5 = wave_max(max_att), c6 = wave_sum(n_defer);
  if (t.lane == 0) {
    if (c0) atomicAdd((unsigned long long *)&a.ctl->stats[DS_COMMITTED], (unsigned long long)c0);
    if (c1) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ATTEMPTS], (unsigned long long)c1);
    if (c2) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_LOCK], (unsigned long long)c2);
    if (c3) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_VALID], (unsigned long long)c3);
    if (c4) atomicAdd((unsigned long long *)&a.ctl->stats[DS_GAVE_UP], (unsigned long long)c4);
    if (c5) atomicMax((unsigned long long *)&a.ctl->stats[DS_MAX_ATTEMPTS], (unsigned long long)c5);
    if (c6) atomicAdd((unsigned long long *)&a.ctl->stats[DS_DEFERRED], (unsigned long long)c6);
  }
}

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
                                                   uint64_t n_aux, DevOutcome *out, uint64_t n_out, Ctl *ctl) {
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
    ctl->ticket = 0;
    ctl->pending_n = 0;
    for (int i = 0; i < DS_N; ++i) ctl->stats[i] = 0;
    ctl->start_clock = wall_clock64();
  }
}

hipError_t launch_init(hipStream_t s, uint64_t *words, uint64_t n_words, uint64_t *aux, uint64_t n_aux,
                       DevOutcome *out, uint64_t n_out, Ctl *ctl) {
  uint64_t n = n_words > n_aux ? n_words : n_aux;
  n = n > n_out ? n : n_out;
  uint64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, words, n_words, aux, n_aux, out, n_out,
                     ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dispatch over (lanes per txn, ops per lane, strict)
// ---------------------------------------------------------------------------
template <int L, int K, int SCHEME, bool STRICT>
static hipError_t launch_one(hipStream_t s, int waves_per_wg, int grid, const RunArgs &a, int n_cu, int *grid_used) {
  auto kern = txn_kernel<L, K, SCHEME, STRICT>;
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

template <int SCHEME, bool STRICT>
static hipError_t dispatch(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, const RunArgs &a,
                           int n_cu, int *grid_used) {
  const int need_k = (max_ops + lanes - 1) / lanes;
#define CCE_TRY(LL, KK)                                                                      \
  if (lanes == LL && need_k <= KK)                                                           \
    return launch_one<LL, KK, SCHEME, STRICT>(s, waves_per_wg, grid, a, n_cu, grid_used);
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

hipError_t launch_txn(hipStream_t s, int scheme, int lanes, int max_ops, int waves_per_wg, int grid, bool strict,
                      const RunArgs &a, int n_cu, int *grid_used) {
  if (scheme != CC_OCC) return hipErrorInvalidValue;
  return strict ? dispatch<CC_OCC, true>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used)
                : dispatch<CC_OCC, false>(s, lanes, max_ops, waves_per_wg, grid, a, n_cu, grid_used);
}

}  // namespace cce
