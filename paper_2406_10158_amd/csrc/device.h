// Device-side building blocks shared by every concurrency-control scheme:
// coherent memory helpers, ordering points, the lane-team abstraction and the
// per-lane operation slots of the transaction a team is executing.
#pragma once

#include "engine.h"

namespace cce {

// ---------------------------------------------------------------------------
// memory helpers: every access to shared state is an agent-scope atomic
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
__device__ __forceinline__ uint64_t and_word(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t add_word(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t xchg_word(uint64_t *p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// compare-and-swap; on failure *expected receives the current value
__device__ __forceinline__ bool cas_word(uint64_t *p, uint64_t *expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_val(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_val(int64_t *p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ordering point: every memory operation issued before it completes before
// any issued after it starts.  The default waits for the wavefront's
// outstanding operations (all shared accesses are coherent atomics, so
// completion is visibility); STRICT adds the agent-scope cache
// write-back/invalidate of a full fence.
template <bool STRICT>
__device__ __forceinline__ void order_point() {
  if constexpr (STRICT) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  } else {
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

// Exclusive prefix sum of v over the wavefront's lanes (lane order); *total
// receives the sum over all lanes.  All lanes must call it.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total) {
  const int lane = __lane_id();
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  *total = (uint32_t)__shfl((int)x, 63, 64);
  return x - v;
}

// A team: the L consecutive lanes (L a power of two) that execute one
// transaction together.
template <int L>
struct Team {
  int lane, tl, tb;  // lane in wave, lane in team, team base lane
  uint64_t tmask;    // this team's lanes
  __device__ __forceinline__ Team() {
    lane = __lane_id();
    tl = lane & (L - 1);
    tb = lane - tl;
    tmask = (L == 64 ? ~0ull : ((1ull << (L & 63)) - 1ull)) << tb;
  }
  // any lane of my team has p
  __device__ __forceinline__ bool any(bool p) const { return (ballot(p) & tmask) != 0; }
  // maximum of v over my team (butterfly within the aligned team block)
  __device__ __forceinline__ uint64_t max(uint64_t v) const {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) {
      uint64_t w = (uint64_t)__shfl_xor((long long)v, o, 64);
      v = w > v ? w : v;
    }
    return v;
  }
  // Teams whose leaders ask (want is uniform per team) share one atomic add
  // of `per` per team on *ctr; returns the counter value before this team's
  // share.  All lanes of the wavefront must call it.
  __device__ __forceinline__ uint64_t claim(uint64_t *ctr, bool want, uint64_t per) const {
    uint64_t m = ballot(want && tl == 0);
    if (m == 0) return 0;
    int first = __ffsll((unsigned long long)m) - 1;
    uint64_t base = 0;
    if (lane == first) base = add_word(ctr, (uint64_t)__popcll(m) * per);
    base = readlane64(base, first);
    uint64_t below = m & ((1ull << tb) - 1ull);
    return base + (uint64_t)__popcll(below) * per;
  }
  // value of v in lane (tb + src_lane)
  __device__ __forceinline__ int64_t shfl(int64_t v, int src_lane) const { return __shfl(v, tb + src_lane, 64); }
};

// ---------------------------------------------------------------------------
// operations
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t op_row(uint32_t rk) { return rk & ROW_MASK; }
__device__ __forceinline__ uint32_t op_kind(uint32_t rk) { return (rk >> KIND_SHIFT) & 3u; }
__device__ __forceinline__ bool op_leader(uint32_t rk) { return !(rk & FOLLOWER_BIT); }
__device__ __forceinline__ bool op_written(uint32_t rk) { return (rk & WRITTEN_BIT) != 0; }

// New value of an operation from its pre-image (operation semantics in cc.h).
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

// Largest workgroup a (lanes, ops-per-lane) variant is compiled for: more
// register slots per lane leave room for fewer wavefronts.
template <int K>
struct MaxThreads {
  static constexpr int value = K <= 1 ? 1024 : (K <= 4 ? 512 : 256);
};

// Per-lane operation slots of the transaction the team executes: lane j of
// the team holds operations j, j+L, ..., j+(K-1)L.
template <int K>
struct Slots {
  uint32_t rowk[K];
  uint32_t elem[K];
  int64_t arg[K];
  uint64_t v[K];  // control word observed / held
  int64_t x[K];   // pre-image read
  uint32_t oi[K]; // op index in the batch
  bool got[K];    // this slot holds its row's lock
  bool valid[K];
  bool sh[K];     // 2PL wait-die: this slot holds a shared lock (kept while the team waits)
  uint32_t block; // a row another transaction held when this attempt failed to lock (~0u: none)
  uint64_t tr[4]; // wall clock at the end of each round (OCC; for the per-round time breakdown)
  uint64_t hot_dt; // OCC: ticks this lane held the batch's most written row in the attempt
  bool hot_got;    // OCC: this lane took that row's lock in the attempt
};

// The first row (in lane order) that a lane of my team found held by another
// transaction, or ~0u.  Team-uniform; every lane of the wavefront must call it.
template <int L>
__device__ __forceinline__ uint32_t blocking_row(const Team<L> &t, uint32_t my_row) {
  const uint64_t m = ballot(my_row != ~0u) & t.tmask;
  if (m == 0) return ~0u;
  const int src = __ffsll((unsigned long long)m) - 1;
  return (uint32_t)__shfl((int)my_row, src, 64);
}

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

// The same for every slot at once, through LDS: each lane writes its read
// values slot-major (row k holds every thread's slot k), then reads each
// WRITE_SLOT source from its lane and slot.  Used at 16 slots per lane, where
// the K x K shuffles of slot_source need more registers than there are.
// Only this wavefront reads what it wrote, and a wavefront's LDS operations
// are performed in order, so wavefront-scope fences suffice.
template <int L, int K>
__device__ __forceinline__ void slot_sources_lds(const Team<L> &t, const Slots<K> &s, int64_t (&src_val)[K]) {
  constexpr int T = MaxThreads<K>::value;
  __shared__ int64_t xs[K * T];
  const int me = (int)threadIdx.x;
  const int team0 = me - t.lane + t.tb;  // thread index of the team's first lane
#pragma unroll
  for (int k = 0; k < K; ++k) xs[k * T + me] = s.x[k];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool slot = s.valid[k] && op_kind(s.rowk[k]) == CC_WRITE_SLOT;
    // a source is an earlier operation of the transaction, so src < L * K
    const uint32_t src = slot ? (uint32_t)(s.arg[k] & 0xFF) : 0u;
    src_val[k] = slot ? xs[(int)(src / L) * T + team0 + (int)(src & (L - 1))] : 0;
  }
  // the next call's writes come after these reads
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Store the new values of a committing team's write operations.  Every lane
// of the wavefront must call it (WRITE_SLOT sources move between lanes).
template <int L, int K>
__device__ __forceinline__ void install_values(const Team<L> &t, const Slots<K> &s, bool commit, const RunArgs &a) {
  if (a.has_slot) {
    int64_t src_val[K];
    if constexpr (K >= 16) {
      slot_sources_lds<L, K>(t, s, src_val);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        uint32_t src = (s.valid[k] && op_kind(s.rowk[k]) == CC_WRITE_SLOT) ? (uint32_t)(s.arg[k] & 0xFF) : 0u;
        src_val[k] = slot_source<L, K>(t, s, src);
      }
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
}

enum AttemptResult { COMMIT = 0, ABORT_LOCK = 1, ABORT_VALID = 2, TS_OVERFLOW = 3, WAITING = 4 };

// Bound on compare-and-swap retries inside one latch-free critical section.
constexpr int CAS_RETRIES = 64;

}  // namespace cce
