// The OCC hot-row engine: the transactions of a batch that write one of its
// most written rows run first, in one workgroup that keeps those rows -- their
// locks, last writers' tickets and values -- in LDS.  The rest of the batch
// then runs in the transaction kernel, where the engine rows are only read.
//
// Why: under skew the batch is serialised on its hottest rows, and on gfx950
// every agent-scope access to a row's word is a round trip to the coherent
// level (about half a microsecond, wherever the wavefronts sit).  OCC holds a
// written row for its ticket, validation and install rounds, and contenders
// that failed on it back off at random, so the row is idle between holders.
// In LDS a lock, a ticket and an install take tens of nanoseconds, and
// contenders can wait for the row instead of backing off.
//
// Protocol (OCC, paper Section 2 "Optimistic Concurrency Control" and Section
// 3.5 "OCC", with the engine rows locked pessimistically -- the hot-record
// locking of mostly-optimistic concurrency control):
//   R1   cold rows exactly as OCC: lock written rows (fetch_or on the word,
//        no wait), load the words of read-only rows; a held row aborts the
//        attempt.  Then the cold values, under the locks / after the words.
//   R1b  engine rows in decreasing engine index, so the most written row
//        (index 0) comes last: a written row takes its LDS lock exclusively,
//        a read-only row shares it.  At the first row that is not free the
//        team gives back every row it took -- engine and cold -- and waits,
//        holding nothing, until that row is free (one LDS load per loop
//        iteration); then it makes a new attempt.  No one waits while holding
//        a row, and a team that holds all of its rows never waits, so every
//        wait ends.
//   R2   the engine rows' values and the ticket, from an LDS counter that
//        starts from the run's ticket counter (the engine runs alone, before
//        the rest of the batch, so its tickets order only its transactions,
//        and the rest draw later ones).  Read-only engine rows are released
//        here: a read under a shared lock is ordered by the ticket drawn
//        while holding it.
//   R3   validation of the cold read-only rows (word unchanged) and of every
//        cold word's ticket (older than ours).
//   R4   engine rows: new values and the ticket into LDS, then the lock
//        released; cold rows: values stored, waited for, then the word set
//        to the ticket (publish + unlock), or restored on failure.
// Serial key (0, ticket), as OCC.  At the end the engine rows' words (their
// last writer's ticket, unlocked) and values go back to the table, and the
// LDS ticket counter to the run's.
#pragma once

#include "schemes.h"

namespace cce {

constexpr uint32_t ENG_WRITER = 1u << 31;  // LDS lock: writer bit; bits 0-30 count readers
static_assert((ENG_MAX & (ENG_MAX - 1)) == 0 && ENG_MAX <= 32, "engine rows: a power of two, one bit each");

// Engine index of `row` (-1: not an engine row) and, for an engine row, the
// LDS index of its cell `elem`.  The loop is unrolled so that every e.*[i]
// is a scalar operand: indexed by a lane's value, the kernel arguments would
// be read from memory.
__device__ __forceinline__ int eng_index(const EngineArgs &e, uint32_t row, uint32_t elem, uint32_t *cell) {
  int r = -1;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < ENG_MAX; ++i) {
    const bool hit = (uint32_t)i < e.n_rows && e.row[i] == row;
    r = hit ? i : r;
    c = hit ? e.off[i] + (elem - e.elem0[i]) : c;
  }
  *cell = c;
  return r;
}

__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// Cold rows in the engine: while the engine runs, only its own workgroup
// touches any row, so the cold rows' locks and versions live in LDS too, in a
// table of ENG_BUCKETS words a row hashes into (rows sharing a bucket share
// its lock: a rare false conflict).  Bucket word: bit 63 locked, bits 47-62
// the locking team, bits 0-46 a version bumped by every commit that writes a
// row of the bucket.  The rows' values stay in global memory; the global
// word of a written row receives the committing ticket (the pass that runs
// after the engine validates against it).
constexpr int ENG_BUCKETS = 16384;
constexpr uint64_t CB_LOCK = 1ull << 63;
constexpr uint64_t CB_VMASK = (1ull << 47) - 1ull;
__device__ __forceinline__ uint32_t cold_bucket(uint32_t row) { return (row * 0x9E3779B1u) >> (32 - 14); }
static_assert(ENG_BUCKETS == 1 << 14, "cold_bucket hashes to 14 bits");
__device__ __forceinline__ uint32_t cb_owner(uint64_t w) { return (uint32_t)((w >> 47) & 0xFFFFu); }

// One attempt of a team (every lane of the wavefront calls it).  WAITING:
// an engine row was taken (*wait_j: which, and ENG_WRITER if to write it);
// the attempt gave back everything it held.
template <int L, int K, bool STRICT>
__device__ __forceinline__ int engine_attempt(const Team<L> &t, Slots<K> &s, const int (&ei)[K],
                                              const uint32_t (&cell)[K], uint32_t emask, bool active,
                                              const RunArgs &a, const EngineArgs &e, uint32_t *lk, uint64_t *tid,
                                              int64_t *val, uint64_t *cb, uint64_t *ticket_ctr, uint64_t *hot_t0,
                                              uint64_t *hot_dt, uint32_t *wait_j, uint64_t *key) {
  bool fail = false;
  uint32_t blk = ~0u;
  const uint32_t me = (uint32_t)threadIdx.x / (uint32_t)L;  // the team in the workgroup
  // R1: the cold rows' buckets -- a written row's locked (no wait), a
  // read-only row's version read (held by another team: abort).  A row's
  // value is loaded as soon as its bucket has been read free (or held by the
  // team itself), so that the load overlaps the lock's round trip: a lock
  // taken with the version read confirms that no commit wrote the row
  // between the two, and a read-only row's version is validated later; a lock
  // that succeeds only after the version moved loads the value again
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    if (active && s.valid[k] && op_leader(s.rowk[k]) && ei[k] < 0) {
      uint64_t *w = cb + cold_bucket(op_row(s.rowk[k]));
      uint64_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      const uint64_t cur0 = cur;
      if (!(cur & CB_LOCK) || cb_owner(cur) == me) s.x[k] = ld_val(a.data + s.elem[k]);
      bool ok = false;
      if (op_written(s.rowk[k])) {
        for (int i = 0; i < 4; ++i) {
          if (cur & CB_LOCK) {
            ok = cb_owner(cur) == me;  // another row of ours in the same bucket
            break;
          }
          if (__hip_atomic_compare_exchange_strong(w, &cur, CB_LOCK | ((uint64_t)me << 47) | (cur & CB_VMASK),
                                                   __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            ok = true;
            s.got[k] = true;
            break;
          }
        }
        if (s.got[k] && cur != cur0) s.x[k] = ld_val(a.data + s.elem[k]);  // the version moved first
      } else {
        ok = !(cur & CB_LOCK) || cb_owner(cur) == me;
      }
      s.v[k] = cur & CB_VMASK;
      if (!ok && blk == ~0u) blk = op_row(s.rowk[k]);
      fail |= !ok;
    }
  }
  const bool lock_fail = t.any(fail);
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) __hip_atomic_store(cb + cold_bucket(op_row(s.rowk[k])), s.v[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  s.block = blocking_row(t, blk);
  lds_fence();  // the buckets before the values
  // the values of rows repeated in the transaction (loaded after their first
  // op's bucket), and every cold value waited for before any engine row is
  // taken, so that no engine row is held across a global round trip
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (active && !lock_fail && s.valid[k] && ei[k] < 0 && !op_leader(s.rowk[k])) s.x[k] = ld_val(a.data + s.elem[k]);
  if (ballot(active && !lock_fail)) order_point<STRICT>();

  // R1b: the engine rows, in decreasing engine index
  const bool go = active && !lock_fail;
  const uint32_t need = go ? emask : 0u;  // team-uniform
  uint32_t held = 0;                      // team-uniform: engine rows taken
  bool stop = false;                      // team-uniform: a row was not free
  uint64_t wneed = 0;
  if (L == 64) {
    // one team per wavefront: its `need` is the wavefront's
    wneed = (uint32_t)__builtin_amdgcn_readfirstlane((int)need);
  } else {
    // rows any team of the wavefront still needs (every lane of a team has `need`)
    uint32_t m = need;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m |= (uint32_t)__shfl_xor((int)m, o, 64);
    wneed = m;
  }
  if constexpr (L == 64 && K == 1) {
    // one team per wavefront and one op per lane: the lane holding an engine
    // row's op takes that row, and the rest of the loop is wavefront-uniform
    const bool eop = go && s.valid[0] && op_leader(s.rowk[0]) && ei[0] >= 0;
    const bool ewr = op_written(s.rowk[0]);
    while (wneed) {
      const int j = 63 - __clzll((unsigned long long)wneed);
      wneed &= ~(1ull << j);
      const bool mine = eop && ei[0] == j;
      bool bad = false;
      if (mine) {
        if (ewr) {
          uint32_t expect = 0;
          bad = !__hip_atomic_compare_exchange_strong(lk + j, &expect, ENG_WRITER, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          const uint32_t old = __hip_atomic_fetch_add(lk + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (old & ENG_WRITER) {
            (void)__hip_atomic_fetch_sub(lk + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            bad = true;
          }
        }
      }
      if (ballot(bad)) {
        stop = true;
        *wait_j = (uint32_t)j | (ballot(mine && ewr) ? ENG_WRITER : 0u);
        break;
      }
      held |= 1u << j;
    }
  }
  while (L < 64 || K > 1 ? wneed : 0) {
    const int j = 63 - __clzll((unsigned long long)wneed);  // wavefront-uniform
    wneed &= ~(1ull << j);
    const bool want = go && !stop && ((need >> j) & 1u);  // team-uniform
    bool tried = false, ok = true, wr = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (want && s.valid[k] && op_leader(s.rowk[k]) && ei[k] == j) {
        tried = true;
        wr = op_written(s.rowk[k]);
        if (wr) {
          uint32_t expect = 0;
          ok = __hip_atomic_compare_exchange_strong(lk + j, &expect, ENG_WRITER, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          const uint32_t old = __hip_atomic_fetch_add(lk + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (old & ENG_WRITER) {
            (void)__hip_atomic_fetch_sub(lk + j, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            ok = false;
          }
        }
      }
    }
    const bool team_fail = t.any(tried && !ok);
    const bool team_wr = t.any(tried && wr);
    if (want) {
      if (team_fail) {
        stop = true;
        *wait_j = (uint32_t)j | (team_wr ? ENG_WRITER : 0u);  // the row waited for, and how
      } else {
        held |= 1u << j;
      }
    }
  }
  lds_fence();  // the locks are taken before anything below reads the rows
  // a team that stopped gives back everything it took: no one waits holding a row
  if (go && stop) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (s.valid[k] && op_leader(s.rowk[k]) && ei[k] >= 0 && ((held >> ei[k]) & 1u)) {
        if (op_written(s.rowk[k]))
          (void)__hip_atomic_fetch_and(lk + ei[k], ~ENG_WRITER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          (void)__hip_atomic_fetch_sub(lk + ei[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (s.got[k])
        __hip_atomic_store(cb + cold_bucket(op_row(s.rowk[k])), s.v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    held = 0;
  }
  // hold statistics of engine row 0 (the batch's most written row), in the
  // lane that writes it: from its lock to its release
  bool w0 = false;
#pragma unroll
  for (int k = 0; k < K; ++k) w0 |= s.valid[k] && op_leader(s.rowk[k]) && op_written(s.rowk[k]) && ei[k] == 0;
  // the time the most written row was taken: read here, collected with the
  // round trip below instead of waited for inside the hold
  const uint64_t t_acq = wall_clock64();
  const bool alive = go && !stop;
  // the engine rows' holders issue first on their SIMD until they release them:
  // the waves polling for those rows share it
  if (ballot(alive)) __builtin_amdgcn_s_setprio(3);

  uint64_t ticket = 0;
  bool valid_fail = false;
  int64_t nv[K];
  if constexpr (L == 64 && K == 1) {
    // one team per wavefront and one op per lane: each lane's part in the hold
    // is decided before it, and the hold runs under one wavefront-uniform branch
    const uint32_t rk = s.rowk[0];
    const bool lead = s.valid[0] && op_leader(rk), wrt = op_written(rk);
    const bool e_op = s.valid[0] && ei[0] >= 0;
    const bool e_rd = e_op && lead && !wrt, e_wr = e_op && lead && wrt;
    const bool c_rd = lead && ei[0] < 0 && !wrt;
    const bool e_inst = e_op && op_kind(rk) != CC_READ;
    const uint32_t src = (a.has_slot && s.valid[0] && op_kind(rk) == CC_WRITE_SLOT) ? (uint32_t)(s.arg[0] & 0xFF) : 0u;
    nv[0] = 0;
    if (ballot(alive)) {
      // R2: engine values and the ticket (one LDS add, collected with the
      // validation loads), read-only engine rows released after the ticket
      if (e_op) s.x[0] = val[cell[0]];
      uint64_t tk = 0;
      if (t.lane == 0)
        tk = __hip_atomic_fetch_add(ticket_ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // LDS operations are performed in issue order
      if (e_rd) (void)__hip_atomic_fetch_sub(lk + ei[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      // R3: the cold read-only rows' buckets unchanged and not held by another team
      bool bad = false;
      if (c_rd) {
        const uint64_t cur = __hip_atomic_load(cb + cold_bucket(op_row(rk)), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
        bad = (((cur & CB_LOCK) != 0) & (cb_owner(cur) != me)) | ((cur & CB_VMASK) != s.v[0]);
      }
      ticket = readlane64(tk, 0) + 1;
      if (w0 && (held & 1u)) *hot_t0 = t_acq;
      valid_fail = ballot(bad) != 0;
      // R4: new values, engine rows installed, then their locks released
      // the new value without branches on the op's kind (WRITE_SLOT only in
      // batches that have slot ops)
      {
        const uint32_t kind = op_kind(rk);
        const int64_t pre = s.x[0];
        const int64_t add = (int64_t)((uint64_t)pre + (uint64_t)s.arg[0]);
        const int64_t cadd = add < CC_COND_LO ? (int64_t)((uint64_t)add + (uint64_t)CC_COND_HI) : add;
        nv[0] = kind == CC_ADD ? add : (kind == CC_COND_ADD ? cadd : pre);
        if (a.has_slot) {
          const int64_t sv = slot_source<L, K>(t, s, src);
          if (kind == CC_WRITE_SLOT) nv[0] = apply_op(CC_WRITE_SLOT, pre, s.arg[0], sv);
        }
      }
      if (!valid_fail && e_inst) val[cell[0]] = nv[0];
      if (!valid_fail && e_wr) tid[ei[0]] = ticket;
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // values and tickets before the locks are free
      if (e_wr) (void)__hip_atomic_fetch_and(lk + ei[0], ~ENG_WRITER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  } else {
    // R2: engine values, the ticket, read-only engine rows released
  #pragma unroll
    for (int k = 0; k < K; ++k)
      if (alive && s.valid[k] && ei[k] >= 0) s.x[k] = val[cell[k]];
    // one LDS add draws the tickets of the wavefront's live teams; its result is
    // collected after the validation loads below are issued, so that both
    // come back in one round trip
    const uint64_t tk_m = ballot(alive && t.tl == 0);
    const int tk_first = __ffsll((unsigned long long)tk_m) - 1;
    uint64_t tk_base = 0;
    if (tk_m && t.lane == tk_first)
      tk_base = __hip_atomic_fetch_add(ticket_ctr, (uint64_t)__popcll(tk_m), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
    // the ticket is drawn before the releases and validation below: a
    // wavefront's LDS operations are performed in the order it issues them, so
    // only the compiler has to keep that order
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  #pragma unroll
    for (int k = 0; k < K; ++k)
      if (alive && s.valid[k] && op_leader(s.rowk[k]) && ei[k] >= 0 && !op_written(s.rowk[k]))
        (void)__hip_atomic_fetch_sub(lk + ei[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);

    // R3: validation of the cold read-only rows: their buckets unchanged and
    // not held by another team
    bool bad = false;
  #pragma unroll
    for (int k = 0; k < K; ++k) {
      if (alive && s.valid[k] && op_leader(s.rowk[k]) && ei[k] < 0 && !op_written(s.rowk[k])) {
        const uint64_t cur = __hip_atomic_load(cb + cold_bucket(op_row(s.rowk[k])), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
        bad |= ((cur & CB_LOCK) && cb_owner(cur) != me) || (cur & CB_VMASK) != s.v[k];
      }
    }
    ticket =
        tk_m ? readlane64(tk_base, tk_first) + 1 + (uint64_t)__popcll(tk_m & ((1ull << t.tb) - 1ull)) : 0;
    if (w0 && go && !stop && (held & 1u)) *hot_t0 = t_acq;
    valid_fail = t.any(bad);
    const bool commit = alive && !valid_fail;

    // R4: new values (WRITE_SLOT sources move between lanes: every lane takes part)
    {
      int64_t src_val[K];
  #pragma unroll
      for (int k = 0; k < K; ++k) {
        uint32_t src = (a.has_slot && s.valid[k] && op_kind(s.rowk[k]) == CC_WRITE_SLOT) ? (uint32_t)(s.arg[k] & 0xFF) : 0u;
        src_val[k] = a.has_slot ? slot_source<L, K>(t, s, src) : 0;
      }
  #pragma unroll
      for (int k = 0; k < K; ++k) nv[k] = apply_op(op_kind(s.rowk[k]), s.x[k], s.arg[k], src_val[k]);
    }
    // engine rows first: their install and release wait for nothing global
  #pragma unroll
    for (int k = 0; k < K; ++k)
      if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ && ei[k] >= 0) val[cell[k]] = nv[k];
  #pragma unroll
    for (int k = 0; k < K; ++k)
      if (alive && s.valid[k] && op_leader(s.rowk[k]) && op_written(s.rowk[k]) && ei[k] >= 0 && commit) tid[ei[k]] = ticket;
    // values and tickets are in LDS before the locks are free (LDS operations
    // of a wavefront are performed in issue order)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  #pragma unroll
    for (int k = 0; k < K; ++k)
      if (alive && s.valid[k] && op_leader(s.rowk[k]) && op_written(s.rowk[k]) && ei[k] >= 0)
        (void)__hip_atomic_fetch_and(lk + ei[k], ~ENG_WRITER, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  const bool commit = alive && !valid_fail;
  __builtin_amdgcn_s_setprio(0);
  if (alive && *hot_t0) *hot_dt = wall_clock64() - *hot_t0;
  // cold rows: values and words to global memory, then the buckets released
  // with a new version (a workgroup-scope release: another wavefront that
  // sees the bucket free and then loads a value reads the new one)
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ && ei[k] < 0) st_val(a.data + s.elem[k], nv[k]);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (commit && s.valid[k] && op_leader(s.rowk[k]) && op_written(s.rowk[k]) && ei[k] < 0)
      st_word(a.words + op_row(s.rowk[k]), ticket);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.got[k])
      __hip_atomic_store(cb + cold_bucket(op_row(s.rowk[k])), commit ? ((s.v[k] + 1) & CB_VMASK) : s.v[k],
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  *key = ticket;
  if (!active) return COMMIT;
  if (lock_fail) return ABORT_LOCK;
  if (stop) return WAITING;
  return valid_fail ? ABORT_VALID : COMMIT;
}

// Looks a waiting wavefront takes at its row before going round its main loop.
constexpr int ENG_SPIN = 64;

// Loads the ops of the staged transaction nx_d into the staging registers.
template <int L, int K>
__device__ __forceinline__ void load_next_ops(const Team<L> &t, const RunArgs &a, const EngineDesc &nx_d,
                                              uint32_t (&nx_rowk)[K], uint32_t (&nx_elem)[K], int64_t (&nx_arg)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
    if (idx < nx_d.n) {
      const DevOp op = a.ops[nx_d.first + idx];
      nx_rowk[k] = op.rowk;
      nx_elem[k] = op.elem;
      nx_arg[k] = op.arg;
    }
  }
}

// A team with no transaction takes the staged one (loading its ops first if
// they are not in registers yet): its slots, engine indices and LDS cells.
template <int L, int K>
__device__ __forceinline__ void take_next(const Team<L> &t, Slots<K> &s, const EngineArgs &e, const RunArgs &a,
                                          int &nx_state, const EngineDesc &nx_d, uint32_t (&nx_rowk)[K],
                                          uint32_t (&nx_elem)[K], int64_t (&nx_arg)[K], int (&ei)[K],
                                          uint32_t (&cell)[K], uint32_t *emask, int64_t *txn, uint32_t *first,
                                          uint32_t *n) {
  if (nx_state == 0) return;
  if (nx_state == 1) load_next_ops<L, K>(t, a, nx_d, nx_rowk, nx_elem, nx_arg);
  *txn = (int64_t)nx_d.txn;
  *first = nx_d.first;
  *n = nx_d.n;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t idx = (uint32_t)t.tl + (uint32_t)(k * L);
    s.valid[k] = idx < nx_d.n;
    s.oi[k] = nx_d.first + idx;
    s.rowk[k] = s.valid[k] ? nx_rowk[k] : FOLLOWER_BIT;
    s.elem[k] = s.valid[k] ? nx_elem[k] : 0u;
    s.arg[k] = s.valid[k] ? nx_arg[k] : 0;
    s.x[k] = 0;
    s.v[k] = 0;
    ei[k] = s.valid[k] ? eng_index(e, op_row(s.rowk[k]), s.elem[k], &cell[k]) : -1;
  }
  // the engine rows the transaction touches come with its descriptor (a
  // wavefront-uniform value when the team is the wavefront)
  *emask = L == 64 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)nx_d.emask) : nx_d.emask;
  nx_state = 0;
}

template <int L, int K, bool STRICT>
__global__ void __launch_bounds__(MaxThreads<K>::value) engine_kernel(RunArgs a, EngineArgs e) {
  __shared__ uint32_t lk[ENG_MAX];
  __shared__ uint64_t tid[ENG_MAX];
  __shared__ int64_t val[ENG_VALS];
  __shared__ uint64_t cb[ENG_BUCKETS];
  __shared__ uint64_t ticket_ctr;
  __shared__ uint32_t queue_ctr;
  const uint32_t me = threadIdx.x, nthr = blockDim.x;
  // the engine rows come into LDS
  for (uint32_t i = me; i < e.n_rows; i += nthr) {
    lk[i] = 0;
    tid[i] = ld_word(a.words + e.row[i]) & ~OCC_LOCK;
  }
  for (uint32_t v = me; v < e.n_vals; v += nthr) {
    uint32_t i = 0;
    while (i + 1 < e.n_rows && e.off[i + 1] <= v) ++i;
    val[v] = ld_val(a.data + e.elem0[i] + (v - e.off[i]));
  }
  for (uint32_t i = me; i < (uint32_t)ENG_BUCKETS; i += nthr) cb[i] = 0;
  if (me == 0) {
    ticket_ctr = ld_word(&a.ctl->ticket);
    queue_ctr = 0;
  }
  __syncthreads();

  Team<L> t;
  Slots<K> s;
  int ei[K];
  uint32_t cell[K];       // an engine op's cell in LDS
  uint32_t emask = 0;     // team-uniform: engine rows the transaction touches
  const uint64_t start_clock = a.ctl->start_clock;
  int64_t txn = -1;
  uint32_t first = 0, n = 0;  // the transaction's ops
  uint32_t attempts = 0;
  uint64_t ready_at = 0;
  uint32_t wait_j = 0;    // team-uniform: the engine row a waiting team stopped at (ENG_WRITER: to write it)
  bool waiting = false;   // the team waits, holding nothing, for engine row wait_j
  // the next transaction (team-uniform): 0 none, 1 descriptor loaded, 2 ops loaded too
  int nx_state = 0;
  bool nx_end = false;    // no transaction left to claim
  EngineDesc nx_d{0, 0, 0, 0};
  uint32_t nx_rowk[K], nx_elem[K];
  int64_t nx_arg[K];
  uint64_t n_commit = 0, n_att = 0, n_lock = 0, n_valid = 0, n_gave = 0, max_att = 0, n_waits = 0;
  uint64_t t_useful = 0, t_abort = 0, t_wait = 0;
  uint64_t n_hot_acq = 0, n_hot_fail = 0, t_hot = 0;
  uint64_t hot_t0 = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ei[k] = -1;
    cell[k] = 0;
  }

  for (;;) {
    // the next transaction is staged while the current one runs: claimed and
    // its descriptor loaded in one iteration, its ops loaded after that
    // iteration's rounds, taken from registers when the current one ends
    if (txn < 0) {
      take_next<L, K>(t, s, e, a, nx_state, nx_d, nx_rowk, nx_elem, nx_arg, ei, cell, &emask, &txn, &first, &n);
      attempts = 0;
      ready_at = 0;
      waiting = false;
    }
    if (nx_state == 0 && !nx_end) {
      uint32_t q = 0;
      const uint64_t m = ballot(t.tl == 0);
      const int lead = __ffsll((unsigned long long)m) - 1;
      uint32_t base = 0;
      if (t.lane == lead)
        base = __hip_atomic_fetch_add(&queue_ctr, (uint32_t)__popcll(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      base = (uint32_t)__builtin_amdgcn_readlane((int)base, lead);
      q = base + (uint32_t)__popcll(m & ((1ull << t.tb) - 1ull));
      if (q < e.n_txns) {
        nx_d = e.desc[q];
        nx_state = 1;
      } else {
        nx_end = true;
      }
    }
    if (txn < 0) {
      // a team with nothing to run (its first transaction): take the one just claimed
      take_next<L, K>(t, s, e, a, nx_state, nx_d, nx_rowk, nx_elem, nx_arg, ei, cell, &emask, &txn, &first, &n);
      attempts = 0;
      ready_at = 0;
      waiting = false;
    }
    if (ballot(txn >= 0) == 0) break;
    uint64_t now = wall_clock64();
    bool active = txn >= 0 && now >= ready_at;
    if (active && waiting) {
      // a waiting team looks only at the row it waits for, and tries again once that row is free
      const uint32_t wj = L == 64 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)wait_j) : wait_j;
      const uint32_t *wl = lk + (wj & (ENG_MAX - 1));
      const bool wr = (wj & ENG_WRITER) != 0;
      uint32_t w = __hip_atomic_load(wl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (L == 64 && (wr ? w != 0 : (w & ENG_WRITER) != 0)) {
        // the wavefront's one team waits: its next transaction's ops are loaded
        // meanwhile, and it looks at the row in a short loop of its own (a
        // bounded number of looks, then once round the main loop)
        if (nx_state == 1) {
          load_next_ops<L, K>(t, a, nx_d, nx_rowk, nx_elem, nx_arg);
          nx_state = 2;
        }
        w = (uint32_t)__builtin_amdgcn_readfirstlane((int)w);
        for (int i = 0; i < ENG_SPIN && (wr ? w != 0 : (w & ENG_WRITER) != 0); ++i) {
          __builtin_amdgcn_s_sleep(1);
          w = (uint32_t)__builtin_amdgcn_readfirstlane(
              (int)__hip_atomic_load(wl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        }
        const uint64_t now2 = wall_clock64();
        if (t.tl == 0) t_wait += now2 - now;
        now = now2;
      }
      active = wr ? w == 0 : !(w & ENG_WRITER);
    }
    if (ballot(active) == 0) {
      if (nx_state == 1) {
        load_next_ops<L, K>(t, a, nx_d, nx_rowk, nx_elem, nx_arg);
        nx_state = 2;
      }
      __builtin_amdgcn_s_sleep(1);
      if (txn >= 0 && t.tl == 0) t_wait += wall_clock64() - now;
      continue;
    }
    uint64_t key = 0, hot_dt = 0;
    // a transaction on the most written row runs ahead of the others on its
    // SIMD (its holders go higher still): its attempts are the batch's critical path
    if (ballot(active && (emask & 1u))) __builtin_amdgcn_s_setprio(2);
    const int r = engine_attempt<L, K, STRICT>(t, s, ei, cell, emask, active, a, e, lk, tid, val, cb, &ticket_ctr,
                                               &hot_t0, &hot_dt, &wait_j, &key);
    if (t.tl == 0 && txn >= 0) {
      const uint64_t dt = wall_clock64() - now;
      if (!active || r == WAITING) t_wait += dt;
      else if (r == COMMIT) t_useful += dt;
      else t_abort += dt;
    }
    if (active && r != WAITING && hot_t0) {
      // this lane held the most written row in the attempt that just ended
      ++n_hot_acq;
      n_hot_fail += r != COMMIT;
      t_hot += hot_dt;
      hot_t0 = 0;
    }
    if (active && r == WAITING) {
      waiting = true;
      if (t.tl == 0) ++n_waits;
      ready_at = now;
    } else if (active) {
      waiting = false;
      ++attempts;
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
          if (r == ABORT_LOCK) ++n_lock;
          else ++n_valid;
        }
        if (attempts >= a.max_attempts) {
          if (t.tl == 0) {
            a.out[txn].attempts = attempts;
            ++n_gave;
            max_att = attempts > max_att ? attempts : max_att;
          }
          txn = -1;
        } else {
          const uint32_t sh = attempts < 12 ? attempts : 12;
          const uint64_t span = (uint64_t)a.backoff_ticks << sh;
          ready_at = now + (mix64(((uint64_t)txn << 20) ^ attempts) % (span + 1));
        }
      }
    }
    // the next transaction's descriptor arrived during this iteration's rounds: its ops now
    if (nx_state == 1) {
      load_next_ops<L, K>(t, a, nx_d, nx_rowk, nx_elem, nx_arg);
      nx_state = 2;
    }
  }

  // the engine rows and the ticket counter go back
  __syncthreads();
  for (uint32_t i = me; i < e.n_rows; i += nthr) st_word(a.words + e.row[i], tid[i]);
  for (uint32_t v = me; v < e.n_vals; v += nthr) {
    uint32_t i = 0;
    while (i + 1 < e.n_rows && e.off[i + 1] <= v) ++i;
    st_val(a.data + e.elem0[i] + (v - e.off[i]), val[v]);
  }
  if (me == 0) st_word(&a.ctl->ticket, ticket_ctr);

  n_att = t.tl == 0 ? n_att : 0;
  const uint64_t c0 = wave_sum(n_commit), c1 = wave_sum(n_att), c2 = wave_sum(n_lock), c3 = wave_sum(n_valid),
                 c4 = wave_sum(n_gave), c5 = wave_max(max_att), c8 = wave_sum(t_useful), c9 = wave_sum(t_abort),
                 c10 = wave_sum(t_wait), c13 = wave_sum(n_waits), c14 = wave_sum(n_hot_acq),
                 c15 = wave_sum(n_hot_fail), c16 = wave_sum(t_hot);
  if (t.lane == 0) {
    if (c0) atomicAdd((unsigned long long *)&a.ctl->stats[DS_COMMITTED], (unsigned long long)c0);
    if (c1) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ATTEMPTS], (unsigned long long)c1);
    if (c2) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_LOCK], (unsigned long long)c2);
    if (c3) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ABORT_VALID], (unsigned long long)c3);
    if (c4) atomicAdd((unsigned long long *)&a.ctl->stats[DS_GAVE_UP], (unsigned long long)c4);
    if (c5) atomicMax((unsigned long long *)&a.ctl->stats[DS_MAX_ATTEMPTS], (unsigned long long)c5);
    if (c8) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_USEFUL], (unsigned long long)c8);
    if (c9) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_ABORT], (unsigned long long)c9);
    if (c10) atomicAdd((unsigned long long *)&a.ctl->stats[DS_T_WAIT], (unsigned long long)c10);
    if (c13) atomicAdd((unsigned long long *)&a.ctl->stats[DS_ENGINE_WAITS], (unsigned long long)c13);
    if (c14) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_ACQ], (unsigned long long)c14);
    if (c15) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_FAILED], (unsigned long long)c15);
    if (c16) atomicAdd((unsigned long long *)&a.ctl->stats[DS_HOT_HOLD], (unsigned long long)c16);
  }
}

template <int L, int K, bool STRICT>
static hipError_t launch_engine_one(hipStream_t s, int waves, const RunArgs &a, const EngineArgs &e,
                                    int *threads_used) {
  int block = MaxThreads<K>::value;
  if (waves > 0 && 64 * waves < block) block = 64 * waves;
  *threads_used = block;
  hipLaunchKernelGGL((engine_kernel<L, K, STRICT>), dim3(1), dim3(block), 0, s, a, e);
  return hipGetLastError();
}

template <bool STRICT>
static hipError_t engine_dispatch(hipStream_t s, int lanes, int max_ops, int waves, const RunArgs &a,
                                  const EngineArgs &e, int *threads_used) {
  const int need_k = (max_ops + lanes - 1) / lanes;
#define CCE_ENG(LL, KK) \
  if (lanes == LL && need_k <= KK) return launch_engine_one<LL, KK, STRICT>(s, waves, a, e, threads_used);
  CCE_ENG(1, 4)
  CCE_ENG(4, 4)
  CCE_ENG(16, 1)
  CCE_ENG(16, 4)
  CCE_ENG(64, 1)
  CCE_ENG(64, 4)
#undef CCE_ENG
  return hipErrorInvalidValue;
}

}  // namespace cce
