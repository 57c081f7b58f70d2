// One execution attempt of a transaction under each concurrency-control
// scheme.  Every function is called by all 64 lanes of a wavefront; `active`
// says whether this lane's team runs an attempt now.  Rounds are
// wavefront-synchronous and separated by ordering points; a team votes on
// abort with a ballot over its lanes.  All schemes are no-wait: a conflict
// aborts the attempt (waiting is unsafe when the holder may be a lane of the
// same wavefront, which cannot make progress while this one spins -- paper
// Section 3.4, "Spin Lock").  Returned through hi/lo: the serial key.
#pragma once

#include "device.h"

namespace cce {

// ---------------------------------------------------------------------------
// Control-word updates.  By default each is one 64-bit atomic on the word
// (the paper's latch-free form, Section 3.5).  With LATCH (CC_RUN_LATCH) a
// 32-bit latch per row guards the word instead, as in the paper's latch
// variants of the schemes (Section 4.2, Exp-7): every write of the word,
// releases included, takes the latch, so each update is a critical section
// [latch, load, store, unlatch] equivalent to the atomic it replaces, and
// plain loads of the word stay valid.  The CAS on the latch, the section and
// the release are one iteration of the spin loop (Section 3.4, "Spin
// Lock"): a lane of the same wavefront that holds the latch finishes its
// section in the iteration it took the latch, so spinning lanes cannot
// block it.
// ---------------------------------------------------------------------------
constexpr uint32_t LATCH_SPINS = 1u << 22;

// A latch that is not obtained within LATCH_SPINS tries fails the run: the
// first team to give up sets the stop word, every later latched update gives
// up at once (it checks the word every 1024 tries), and the persistent loop
// of every team exits at its next iteration.  An update that gave up is not
// applied; it returns the word with bit 63 set, which every scheme reads as
// "held" (OCC / TicToc lock, 2PL exclusive, TO dirty), so acquisitions and
// compare-and-swaps fail and their attempts abort.  A lost release leaves its
// row held, and cc_run reports CC_E_LIVELOCK with the table contents
// undefined.
template <bool STRICT, class F>
__device__ __forceinline__ uint64_t latched(const RunArgs &a, uint64_t *w, F f) {
  uint32_t *lt = a.latch + (w - a.words);
  for (uint32_t it = 0; it < LATCH_SPINS; ++it) {
    if (it && (it & 1023u) == 0 && ld_word(&a.ctl->stop)) return ld_word(w) | (1ull << 63);
    uint32_t e = 0;
    if (__hip_atomic_compare_exchange_strong(lt, &e, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      const uint64_t old = ld_word(w);
      const uint64_t nw = f(old);
      if (nw != old) st_word(w, nw);
      order_point<STRICT>();  // the word's new value is performed before the latch is free
      __hip_atomic_store(lt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return old;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  // a latch no one released in 2^22 tries: the run fails
  add_word(&a.ctl->stats[DS_LATCH_STUCK], 1ull);
  st_word(&a.ctl->stop, 1ull);
  return ld_word(w) | (1ull << 63);
}

template <bool LATCH, bool STRICT>
__device__ __forceinline__ uint64_t w_or(const RunArgs &a, uint64_t *w, uint64_t v) {
  if constexpr (LATCH) return latched<STRICT>(a, w, [&](uint64_t o) { return o | v; });
  else return or_word(w, v);
}
template <bool LATCH, bool STRICT>
__device__ __forceinline__ uint64_t w_and(const RunArgs &a, uint64_t *w, uint64_t v) {
  if constexpr (LATCH) return latched<STRICT>(a, w, [&](uint64_t o) { return o & v; });
  else return and_word(w, v);
}
template <bool LATCH, bool STRICT>
__device__ __forceinline__ uint64_t w_add(const RunArgs &a, uint64_t *w, uint64_t v) {
  if constexpr (LATCH) return latched<STRICT>(a, w, [&](uint64_t o) { return o + v; });
  else return add_word(w, v);
}
template <bool LATCH, bool STRICT>
__device__ __forceinline__ bool w_cas(const RunArgs &a, uint64_t *w, uint64_t *expected, uint64_t desired) {
  if constexpr (LATCH) {
    const uint64_t want = *expected;
    const uint64_t old = latched<STRICT>(a, w, [&](uint64_t o) { return o == want ? desired : o; });
    *expected = old;
    return old == want;
  } else {
    return cas_word(w, expected, desired);
  }
}
template <bool LATCH, bool STRICT>
__device__ __forceinline__ void w_st(const RunArgs &a, uint64_t *w, uint64_t v) {
  if constexpr (LATCH) (void)latched<STRICT>(a, w, [&](uint64_t) { return v; });
  else st_word(w, v);
}

// An update whose kind is data: one call site, and so one spin loop, serves
// lanes that need different updates at the same program point.  With LATCH
// this matters for forward progress: when two sibling branches each took a
// latch, the compiler may hoist their identical latch CAS above the branch,
// so a lane of one branch holds its latch while masked off until the other
// branch's spin loop has finished -- and a lane of that loop spinning on the
// same latch never gets it.  Returns the word before the update; WOP_CAS
// (x = expected, y = desired) succeeded iff the result equals x.
enum WordOp : uint32_t { WOP_ADD = 0, WOP_AND = 1, WOP_CAS = 2 };

template <bool LATCH, bool STRICT>
__device__ __forceinline__ uint64_t w_apply(const RunArgs &a, uint64_t *w, uint32_t op, uint64_t x, uint64_t y) {
  if constexpr (LATCH) {
    return latched<STRICT>(a, w, [&](uint64_t o) {
      return op == WOP_ADD ? o + x : (op == WOP_AND ? (o & x) : (o == x ? y : o));
    });
  } else {
    if (op == WOP_ADD) return add_word(w, x);
    if (op == WOP_AND) return and_word(w, x);
    uint64_t e = x;
    (void)cas_word(w, &e, y);
    return e;
  }
}

// ===========================================================================
// OCC, Silo-style (paper Section 2 "Optimistic Concurrency Control";
// Section 3.5 "OCC"; control word per row = lock bit + 63-bit TID, Table 2).
//
//   R1  write rows: try-lock with fetch_or(LOCK); the returned word is the
//       row's committed TID, a set lock bit means it is held -> abort.
//       read-only rows: load the TID word; locked -> abort.
//   R2  read every operation's value (write rows under our lock) and draw the
//       serial ticket, which is also the TID our writes will carry.
//   R3  validate: each read-only row still has the observed word, and every
//       observed TID is older than our ticket; then store the new values
//       and wait.  (CC_RUN_EAGER_INSTALL stores them in the validation round
//       instead, and stores the pre-images back on a failed validation.)
//   R4  store word = ticket on each write row: publishes the values and
//       releases the lock in one store.  A failed attempt restores the old
//       word -- or, after an eager install, also publishes its ticket, so
//       that anyone who read a value it stored fails validation.
// The paper's Silo locks the write set at validation time, after its read
// phase.  Read/write sets here are known before execution (Section 4.1,
// "Constraints"), so write rows are locked first and read under the lock,
// which shortens the time a hot row is held or exposed to invalidation.
// Serial key (0, ticket): tickets are drawn while every write lock is held
// and before validation, so conflicting transactions are ordered by ticket.
// ===========================================================================
constexpr uint64_t OCC_LOCK = 1ull << 63;

// True if `row` is one of the batch's hot rows (RunArgs::late).
__device__ __forceinline__ bool is_late(const RunArgs &a, uint32_t row) {
  bool r = false;
#pragma unroll
  for (int i = 0; i < HOT_MAX; ++i) r |= (uint32_t)i < a.n_late && a.late[i] == row;
  return r;
}

// True if this lane holds the lock of the batch's most written row.
template <int K>
__device__ __forceinline__ bool holds_hot0(const Slots<K> &s, const RunArgs &a) {
  bool h = false;
#pragma unroll
  for (int k = 0; k < K; ++k) h |= s.got[k] && op_row(s.rowk[k]) == a.hot0;
  return h;
}

template <int L, int K, bool STRICT, bool LATCH>
__device__ __forceinline__ int occ_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                           bool precheck, uint64_t *hi, uint64_t *lo) {
  bool fail = false;
  uint32_t blk = ~0u;
  bool pre_fail = false;
  s.hot_dt = 0;
  s.hot_got = false;
  // Hot rows last (RunArgs::late): when any team of the wavefront touches one
  // of the batch's hot rows, the lock round is split.  R1 takes every other
  // row; R1b, once those are all held, takes the hot rows.  A hot row is then
  // held only from R1b to R4, and never by an attempt that fails on another
  // row's lock.
  // Not with one lane per transaction, nor in the 16-slot variants: the one
  // run of the split rounds with one lane and 16 slots faulted the GPU, with
  // no out-of-bounds access found in the source, so those variants keep one
  // lock round.
  constexpr bool SPLIT_OK = K < 16 && L > 1;
  bool late[K];
  bool has_late = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    late[k] = SPLIT_OK && active && s.valid[k] && a.n_late && is_late(a, op_row(s.rowk[k]));
    has_late |= late[k];
  }
  const bool split = SPLIT_OK && ballot(has_late) != 0;  // wavefront-uniform
  if (ballot(active && precheck)) {
    // R0, on retries of a contended batch (cc.h, CC_RUN_PRECHECK): load
    // every row's word and give up before taking any lock if one is held, so
    // that failing attempts never hold rows (or write their lines) while
    // they fail elsewhere.  Read-only rows keep the word loaded here, exactly
    // as R1 would load it.  First attempts skip it: until a transaction has
    // failed there is no sign of contention.
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (active && precheck && s.valid[k] && op_leader(s.rowk[k])) {
        const uint64_t o = ld_word(a.words + op_row(s.rowk[k]));
        s.v[k] = o;
        if ((o & OCC_LOCK) && blk == ~0u) blk = op_row(s.rowk[k]);
        fail |= (o & OCC_LOCK) != 0;
      }
    }
    order_point<STRICT>();
    pre_fail = t.any(fail);
  }
  const bool go = active && !pre_fail;
  // R1: locks of written rows, words of read-only rows (hot rows excluded
  // when split).  A split round after R0 also loads these rows' values: a
  // read-only row's value comes after the word R0 saw, which R3 validates; a
  // written row's value is issued beside its lock, and is the row's value
  // under the lock if the lock returns exactly the word R0 saw, unlocked --
  // every commit changes the word to a new ticket for good, and a writer
  // whose install the load could have seen held the lock from before the
  // load until after its new ticket was stored.  A lock that returns another
  // word fails the attempt.
  // The round issues every lock and load first and looks at the results
  // only after the ordering point: a wavefront whose lanes both lock and load
  // then waits for one round trip, not for the locks' and the loads' in turn.
  const bool early_vals = split && precheck;
  bool issued[K];
  uint64_t seen[K];  // the word R0 saw (early_vals)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    seen[k] = s.v[k];
    issued[k] = go && s.valid[k] && op_leader(s.rowk[k]) && !late[k] && (!precheck || op_written(s.rowk[k]));
    if (issued[k]) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      if (op_written(s.rowk[k])) s.v[k] = w_or<LATCH, STRICT>(a, w, OCC_LOCK);
      else s.v[k] = ld_word(w);
    }
    if (early_vals && go && s.valid[k] && !late[k]) s.x[k] = ld_val(a.data + s.elem[k]);
  }
  order_point<STRICT>();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!issued[k]) continue;
    const uint64_t o = s.v[k];
    if ((o & OCC_LOCK) && blk == ~0u) blk = op_row(s.rowk[k]);
    if (op_written(s.rowk[k])) {
      s.got[k] = !(o & OCC_LOCK);
      fail |= !s.got[k] || (early_vals && o != seen[k]);
    } else {
      fail |= (o & OCC_LOCK) != 0;
    }
  }
  s.tr[0] = wall_clock64();
  uint64_t hot_t0 = holds_hot0(s, a) ? s.tr[0] : 0;
  bool lock_fail = t.any(fail);
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
  }
  if (split) {
    // R1b: the hot rows, once every other row is held; without R0 also the
    // other rows' values (under their locks, after their words)
    const bool go2 = active && !lock_fail;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      issued[k] = go2 && op_leader(s.rowk[k]) && late[k];
      if (issued[k]) {
        uint64_t *w = a.words + op_row(s.rowk[k]);
        if (op_written(s.rowk[k])) s.v[k] = w_or<LATCH, STRICT>(a, w, OCC_LOCK);
        else s.v[k] = ld_word(w);
      }
      if (go2 && !precheck && s.valid[k] && !late[k]) s.x[k] = ld_val(a.data + s.elem[k]);
    }
    order_point<STRICT>();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!issued[k]) continue;
      const uint64_t o = s.v[k];
      if ((o & OCC_LOCK) && blk == ~0u) blk = op_row(s.rowk[k]);
      if (op_written(s.rowk[k])) s.got[k] = !(o & OCC_LOCK);
      fail |= (o & OCC_LOCK) != 0;
    }
    s.tr[0] = wall_clock64();
    if (!hot_t0 && holds_hot0(s, a)) hot_t0 = s.tr[0];
    const bool fail_b = t.any(fail);
    if (active && fail_b && !lock_fail) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
    }
    lock_fail = fail_b;
  }
  s.block = blocking_row(t, blk);
  const bool alive = active && !lock_fail;
  if (hot_t0 && !alive) {
    s.hot_got = true;
    s.hot_dt = wall_clock64() - hot_t0;
  }
  // R2: values under the locks / after the observed words (only the hot
  // rows' when split), and the ticket
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.valid[k] && (!split || late[k])) s.x[k] = ld_val(a.data + s.elem[k]);
  const uint64_t ticket = t.claim(&a.ctl->ticket, alive, 1) + 1;
  order_point<STRICT>();
  s.tr[1] = wall_clock64();
  // R3: validation loads (with CC_RUN_EAGER_INSTALL also the new values,
  // stored under the write locks in the same round)
  bool bad = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (alive && s.valid[k] && op_leader(s.rowk[k])) {
      if (!op_written(s.rowk[k])) bad |= ld_word(a.words + op_row(s.rowk[k])) != s.v[k];
      bad |= (s.v[k] & ~OCC_LOCK) >= ticket;
    }
  }
  const bool eager = a.eager_install != 0;
  if (eager) install_values<L, K>(t, s, alive, a);
  const bool valid_fail = t.any(bad);
  const bool commit = alive && !valid_fail;
  if (!eager) install_values<L, K>(t, s, commit, a);
  order_point<STRICT>();
  s.tr[2] = wall_clock64();
  if (eager && alive && valid_fail) {
    // undo: put the pre-images back, and wait for them before the words
    // are released
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.valid[k] && op_kind(s.rowk[k]) != CC_READ) st_val(a.data + s.elem[k], s.x[k]);
  }
  if (eager && ballot(alive && valid_fail)) order_point<STRICT>();
  // R4: one store per write row publishes the values and releases the lock.
  // An aborted attempt also publishes its ticket as the row's TID: its values
  // were visible under the lock, so a reader that saw them must fail
  // validation, which a restored old TID would not guarantee.
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), (commit || eager) ? ticket : s.v[k]);
  s.tr[3] = wall_clock64();
  if (hot_t0 && alive) {
    s.hot_got = true;
    s.hot_dt = s.tr[3] - hot_t0;
  }
  *hi = 0;
  *lo = ticket;
  if (!active) return COMMIT;
  return lock_fail ? ABORT_LOCK : (valid_fail ? ABORT_VALID : COMMIT);
}

// ===========================================================================
// Two-phase locking, no-wait (paper Section 2 "Two-Phase Locking"; Section
// 3.5 "Two-Phase Locking"; lock word = shared-mode bit, 31-bit holder
// count, 31-bit holder, Table 2).  Layout here: bit 63 exclusive, bits 62-32
// holder (transaction id), bits 30-0 shared-holder count.
//   R1  exclusive rows: CAS 0 -> EXCL|holder; shared rows: fetch_add(1) and
//       abort if the exclusive bit was set (the increment is undone).
//   R2  read values under the locks; draw the ticket at the lock point.
//   R3  store new values, wait, release (clear exclusive bits with fetch_and,
//       so concurrent failed shared increments are not lost; fetch_add(-1)).
// Serial key (0, ticket): strict 2PL, ticket drawn while all locks are held.
// ===========================================================================
constexpr uint64_t TPL_EXCL = 1ull << 63;
constexpr uint64_t TPL_COUNT = (1ull << 31) - 1ull;

template <int L, int K, bool STRICT, bool LATCH>
__device__ __forceinline__ int tpl_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                           uint32_t txn, uint64_t *hi, uint64_t *lo) {
  bool fail = false;
  uint32_t blk = ~0u;
  bool shared[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    shared[k] = false;
    if (active && s.valid[k] && op_leader(s.rowk[k])) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      // exclusive: CAS 0 -> EXCL|holder; shared: add one holder
      const bool wr = op_written(s.rowk[k]);
      const uint64_t old = w_apply<LATCH, STRICT>(a, w, wr ? WOP_CAS : WOP_ADD, wr ? 0ull : 1ull,
                                                  TPL_EXCL | ((uint64_t)(txn & 0x7FFFFFFFu) << 32));
      shared[k] = !wr;  // a shared increment is in the word until we take it out
      s.got[k] = wr ? old == 0 : !(old & TPL_EXCL);
      if (!s.got[k] && (!wr || (old & TPL_EXCL)) && blk == ~0u) blk = op_row(s.rowk[k]);
      fail |= !s.got[k];
    }
  }
  order_point<STRICT>();
  s.block = blocking_row(t, blk);
  const bool lock_fail = t.any(fail);
  const bool alive = active && !lock_fail;
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      if (shared[k] || s.got[k])
        (void)w_apply<LATCH, STRICT>(a, w, shared[k] ? WOP_ADD : WOP_AND, shared[k] ? ~0ull : TPL_COUNT, 0);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.valid[k]) s.x[k] = ld_val(a.data + s.elem[k]);
  const uint64_t ticket = t.claim(&a.ctl->ticket, alive, 1) + 1;
  order_point<STRICT>();
  install_values<L, K>(t, s, alive, a);
  order_point<STRICT>();
  if (alive) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      if (shared[k] || s.got[k])
        (void)w_apply<LATCH, STRICT>(a, w, shared[k] ? WOP_ADD : WOP_AND, shared[k] ? ~0ull : TPL_COUNT, 0);
    }
  }
  *hi = 0;
  *lo = ticket;
  if (!active) return COMMIT;
  return lock_fail ? ABORT_LOCK : COMMIT;
}

// ===========================================================================
// Two-phase locking, wait-die (paper Section 2 "Two-Phase Locking": a
// transaction that finds a lock held waits if it is older than the holder
// and dies -- aborts -- if it is younger; Section 3.5 implements tpl_nw and
// tpl_wd over the same lock word, Table 2).  Same word and rounds as the
// no-wait form above; the age of a transaction is its index in the batch
// (smaller = older), kept across its restarts, so every transaction is
// eventually the oldest and cannot starve.
//   R1  take the locks not yet held.  A failure on a row held exclusively by
//       a younger transaction means wait: the attempt returns WAITING with
//       every lock it got still held, and the team retries the missing ones
//       on a later iteration of the persistent loop.  Any other failure (a
//       younger requester, readers in the way, or the attempt's waits used
//       up) means die: release everything and abort.
//   R2, R3 as no-wait.
// Waiting only along older-to-younger edges keeps the waits-for graph
// acyclic, and the youngest holder never waits, so some transaction always
// finishes.  The wait is a state of the team in the persistent loop, not a
// spin: the loop keeps running every other team of the wavefront, so a
// holder in the same wavefront is not starved (Section 3.4, "Spin Lock"),
// and the holder keeps its lock while the waiter waits, so the two do not
// retry in lockstep.  Serial key (0, ticket) as 2PL.
// ===========================================================================
template <int L, int K, bool STRICT, bool LATCH>
__device__ __forceinline__ int tplwd_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                             uint32_t txn, bool resume, bool may_wait, uint64_t *hi,
                                             uint64_t *lo) {
  bool die = false, wait = false;
  uint32_t blk = ~0u;
  const uint64_t me = txn & 0x7FFFFFFFu;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!resume) {
      s.got[k] = false;
      s.sh[k] = false;
    }
    if (active && s.valid[k] && op_leader(s.rowk[k]) && !s.got[k]) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      uint64_t seen = 0;
      const bool wr = op_written(s.rowk[k]);
      seen = w_apply<LATCH, STRICT>(a, w, wr ? WOP_CAS : WOP_ADD, wr ? 0ull : 1ull, TPL_EXCL | (me << 32));
      s.got[k] = wr ? seen == 0 : !(seen & TPL_EXCL);
      s.sh[k] = !wr && s.got[k];
      if (!wr && !s.got[k]) (void)w_apply<LATCH, STRICT>(a, w, WOP_ADD, ~0ull, 0);  // take the increment back out
      if (!s.got[k]) {
        if (blk == ~0u) blk = op_row(s.rowk[k]);
        const uint64_t holder = (seen >> 32) & 0x7FFFFFFFu;
        const bool can_wait = may_wait && (seen & TPL_EXCL) && me < holder;
        wait |= can_wait;
        die |= !can_wait;
      }
    }
  }
  order_point<STRICT>();
  s.block = blocking_row(t, blk);
  const bool any_die = t.any(die);
  const bool any_wait = !any_die && t.any(wait);
  if (active && any_die) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!s.got[k]) continue;
      uint64_t *w = a.words + op_row(s.rowk[k]);
      (void)w_apply<LATCH, STRICT>(a, w, s.sh[k] ? WOP_ADD : WOP_AND, s.sh[k] ? ~0ull : TPL_COUNT, 0);
      s.got[k] = false;
      s.sh[k] = false;
    }
  }
  const bool alive = active && !any_die && !any_wait;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (alive && s.valid[k]) s.x[k] = ld_val(a.data + s.elem[k]);
  const uint64_t ticket = t.claim(&a.ctl->ticket, alive, 1) + 1;
  order_point<STRICT>();
  install_values<L, K>(t, s, alive, a);
  order_point<STRICT>();
  if (alive) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!s.got[k]) continue;
      uint64_t *w = a.words + op_row(s.rowk[k]);
      (void)w_apply<LATCH, STRICT>(a, w, s.sh[k] ? WOP_ADD : WOP_AND, s.sh[k] ? ~0ull : TPL_COUNT, 0);
    }
  }
  *hi = 0;
  *lo = ticket;
  if (!active) return COMMIT;
  return any_die ? ABORT_LOCK : (any_wait ? WAITING : COMMIT);
}

// ===========================================================================
// Basic timestamp ordering, and its multi-version form (paper Section 2
// "Timestamp Ordering" and "MVCC"; Section 3.5 "Basic TO" and "MVCC";
// word = commit/dirty bit, 31-bit RTS, 31-bit WTS, Table 2; MVCC adds a
// 64-bit version pointer per row).  Layout: bit 63 dirty (an uncommitted
// write holds the row), bits 61-31 RTS, bits 30-0 WTS.
//   R0  draw a timestamp ts for this attempt (one global counter).
//   R1  write rows: CAS loop -- abort if dirty or ts < RTS or ts < WTS, else
//       set dirty.  read rows: CAS loop -- abort if dirty (no waiting for the
//       writer) or ts < WTS (TO; MVCC instead reads an older version); else
//       raise RTS to ts.
//   R2  read values (MVCC, older version: also the version pointer).
//   R3  re-check read rows: not dirty and the same WTS, so the value read
//       belongs to the version checked in R1.  MVCC old-version reads walk
//       the version chain back to the newest writer with timestamp <= ts.
//   R4  (MVCC: record each write's pre-image in its history node and link
//       it) store new values, wait, publish word = {RTS=ts, WTS=ts}.
// Serial key (0, ts).  Timestamps are relative to the run and must stay
// below 2^31; reaching it stops the run with CC_E_TS_OVERFLOW.
// Version arena (MVCC): a ring of n_nodes slots of 4 words {tag, prev,
// writer ts | cell << 32, pre-image}.  A committing writer takes one slot per
// written field from the ring counter (position pos: slot pos % n_nodes, lap
// gen = pos / n_nodes + 1) and claims it by CAS on the tag, from an idle
// (even) tag of an earlier lap to 2gen-1 (writing), and stores 2gen once the
// node is written.  A version pointer (the row's, or a node's prev) is gen << 32 |
// (slot + 1); 0 is none.  A chain lists a row's writers newest first; a
// reader at ts starts from the current value and undoes, field by field,
// every writer newer than ts.  It reads a node's fields, then its tag: a tag
// other than 2gen means the slot was taken again by a later lap, so the
// version is gone and the attempt aborts (its retry draws a newer ts).  A
// node is complete before any reader can reach it: it is linked while its
// writer holds the row dirty, and readers walk only chains they found clean
// and unchanged in R3.  The ring is sized by the run: one slot per op of the
// batch, or, when serving, hbm_cap_bytes / 32, which bounds the arena.
// Each run starts with empty chains, so with a slot for every op of the batch
// no slot is ever taken twice in a run: op i then writes its node into slot i
// with no claim and no tag, and readers skip the tag check (node_reuse = 0).
// The claim, the tags and the check are the ring's (node_reuse = 1), for an
// arena smaller than the batch.
// ===========================================================================
constexpr uint64_t TO_DIRTY = 1ull << 63;
constexpr uint64_t TO_MASK31 = (1ull << 31) - 1ull;
__device__ __forceinline__ uint64_t to_rts(uint64_t w) { return (w >> 31) & TO_MASK31; }
__device__ __forceinline__ uint64_t to_wts(uint64_t w) { return w & TO_MASK31; }
__device__ __forceinline__ uint64_t to_word(uint64_t rts, uint64_t wts) { return (rts << 31) | wts; }
constexpr int MVCC_MAX_WALK = 1 << 16;

template <int L, int K, bool STRICT, bool MV, bool LATCH>
__device__ __forceinline__ int to_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                          bool precheck, uint64_t *hi, uint64_t *lo) {
  uint32_t blk = ~0u;
  bool pre_fail = false;
  if (ballot(active && precheck)) {
    // R0 (as OCC's, by default from a transaction's second attempt on): give
    // up before taking a timestamp or marking any row if a row is dirty (an
    // uncommitted write holds it), which R1 would abort on anyway
    bool busy = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (active && precheck && s.valid[k] && op_leader(s.rowk[k])) {
        const uint64_t o = ld_word(a.words + op_row(s.rowk[k]));
        if ((o & TO_DIRTY) && blk == ~0u) blk = op_row(s.rowk[k]);
        busy |= (o & TO_DIRTY) != 0;
      }
    }
    order_point<STRICT>();
    pre_fail = t.any(busy);
  }
  const bool go = active && !pre_fail;
  const uint64_t ts = t.claim(&a.ctl->ticket, go, 1) + 1;
  const bool overflow = go && ts > TO_MASK31;
  bool fail = overflow || (active && pre_fail);
  bool old_ver[K];  // MVCC: this op reads a version older than the current one
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    old_ver[k] = false;
    const bool lead = op_leader(s.rowk[k]);
    // MVCC followers of read rows also look at the word, to pick the version
    const bool look = lead || (MV && !op_written(s.rowk[k]));
    if (go && !overflow && s.valid[k] && look) {
      uint64_t *wp = a.words + op_row(s.rowk[k]);
      uint64_t w = ld_word(wp);
      bool done = false, bad = false;
      for (int it = 0; it < CAS_RETRIES && !done && !bad; ++it) {
        // a write marks the row dirty, a read raises RTS to ts: either way
        // one CAS, issued from a single site (see w_apply)
        bool try_cas = false;
        uint64_t desired = 0;
        if (w & TO_DIRTY) {
          bad = true;
        } else if (op_written(s.rowk[k])) {
          if (ts < to_rts(w) || ts < to_wts(w)) {
            bad = true;
          } else {
            try_cas = true;
            desired = w | TO_DIRTY;
          }
        } else if (ts < to_wts(w)) {
          if (MV) {
            old_ver[k] = true;
            done = true;
          } else {
            bad = true;
          }
        } else if (!lead || to_rts(w) >= ts) {
          done = true;
        } else {
          try_cas = true;
          desired = to_word(ts, to_wts(w));
        }
        if (try_cas && w_cas<LATCH, STRICT>(a, wp, &w, desired)) {
          done = true;
          s.got[k] = op_written(s.rowk[k]);
        }
      }
      s.v[k] = w;
      if ((w & TO_DIRTY) && bad && blk == ~0u) blk = op_row(s.rowk[k]);
      fail |= bad || !done;
    }
  }
  order_point<STRICT>();
  s.block = blocking_row(t, blk);
  const bool lock_fail = t.any(fail);
  const bool alive = active && !lock_fail;
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
  }
  uint64_t ptr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ptr[k] = 0;
    if (alive && s.valid[k]) {
      s.x[k] = ld_val(a.data + s.elem[k]);
      if (MV && old_ver[k]) ptr[k] = ld_word(a.aux + op_row(s.rowk[k]));
    }
  }
  order_point<STRICT>();
  bool bad = false;
  bool same[K];  // the row's word did not change between R1 and R3
#pragma unroll
  for (int k = 0; k < K; ++k) {
    same[k] = true;
    const bool look = op_leader(s.rowk[k]) || (MV && !op_written(s.rowk[k]));
    if (alive && s.valid[k] && look && !op_written(s.rowk[k])) {
      const uint64_t w2 = ld_word(a.words + op_row(s.rowk[k]));
      same[k] = !(w2 & TO_DIRTY) && to_wts(w2) == to_wts(s.v[k]);
      bad |= !same[k];
    }
  }
  if (MV) {
    // Old-version reads walk the chain from the pointer read in R2.  Only
    // when the word did not change: then no writer linked nodes before our
    // R3 load, and writers after it link above that pointer, so the nodes
    // walked are complete.  Indices and length are still bounded.
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (alive && old_ver[k] && same[k]) {
        const uint32_t cell = s.elem[k];
        int64_t val = s.x[k];
        uint64_t p = ptr[k];
        int steps = 0;
        bool gone = false;
        while (p != 0 && steps < MVCC_MAX_WALK) {
          const uint64_t slot = (p & 0xFFFFFFFFull) - 1, gen = p >> 32;
          if (slot >= a.n_nodes) {
            gone = true;
            break;
          }
          const uint64_t *node = a.nodes + 4 * slot;
          const uint64_t prev = ld_word(node + 1), tf = ld_word(node + 2), pre = ld_word(node + 3);
          if (a.node_reuse) {
            order_point<STRICT>();
            // the fields belong to this version only if the slot still carries its tag
            if (ld_word(node) != 2 * gen) {
              gone = true;
              break;
            }
          }
          if ((tf & 0xFFFFFFFFull) <= ts) break;
          if ((uint32_t)(tf >> 32) == cell) val = (int64_t)pre;
          p = prev;
          ++steps;
        }
        if (gone) add_word(&a.ctl->stats[DS_VERSION_MISS], 1ull);
        if (gone || steps >= MVCC_MAX_WALK) bad = true;
        s.x[k] = val;
      }
    }
  }
  bool valid_fail = t.any(bad);
  bool commit = alive && !valid_fail;
  uint64_t pos[K];
  if (MV && !a.node_reuse) {
    // a slot per op: op i's node is slot i, in lap 1
#pragma unroll
    for (int k = 0; k < K; ++k) pos[k] = (uint64_t)s.oi[k];
  } else if (MV) {
    // claim a slot of the version ring for every write op of the committing
    // teams: one fetch_add per wavefront, then a CAS on each slot's tag
    uint32_t nw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) nw += commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ;
    uint32_t total = 0;
    const uint32_t before = wave_excl_scan(nw, &total);
    uint64_t base = 0;
    bool claim_fail = false;
    bool claimed[K];
    if (total) {
      const int first = __ffsll((unsigned long long)ballot(nw != 0)) - 1;
      if (t.lane == first) base = add_word(a.node_ring, (uint64_t)total);
      base = readlane64(base, first);
      uint32_t j = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        claimed[k] = false;
        pos[k] = 0;
        if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ) {
          pos[k] = base + before + j++;
          // any idle tag of an older lap will do (a lap whose claim failed
          // left its older tag behind); an odd tag is a writer at work
          const uint64_t gen = pos[k] / a.n_nodes + 1;
          uint64_t *tag = a.nodes + 4 * (pos[k] % a.n_nodes);
          uint64_t seen = 2 * (gen - 1);
          for (int i = 0; i < 4 && !claimed[k]; ++i) {
            if ((seen & 1) || seen >= 2 * gen) break;
            claimed[k] = cas_word(tag, &seen, 2 * gen - 1);
          }
          claim_fail |= !claimed[k];
        }
      }
      order_point<STRICT>();
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) claimed[k] = false;
    }
    // a slot still being written by a writer of an earlier lap fails the
    // commit: the slots taken are marked done for this lap, holding no
    // version (nothing links to them), and the attempt aborts
    if (t.any(claim_fail) && commit) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (claimed[k]) st_word(a.nodes + 4 * (pos[k] % a.n_nodes), 2 * (pos[k] / a.n_nodes + 1));
      commit = false;
      valid_fail = true;
    }
  }
  if (alive && valid_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
  }
  if (MV) {
    // link each claimed node into its row's chain (we hold the row dirty, so
    // only our own lanes link it concurrently) and fill it; the tag that
    // validates it is stored with the installs, before the row is published
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ) {
        uint64_t *node = a.nodes + 4 * (pos[k] % a.n_nodes);
        const uint64_t me = ((pos[k] / a.n_nodes + 1) << 32) | (pos[k] % a.n_nodes + 1);
        st_word(node + 2, ts | ((uint64_t)s.elem[k] << 32));
        st_word(node + 3, (uint64_t)s.x[k]);
        const uint64_t prev = xchg_word(a.aux + op_row(s.rowk[k]), me);
        st_word(node + 1, prev);
      }
    }
    if (a.node_reuse) {
      order_point<STRICT>();
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (commit && s.valid[k] && op_kind(s.rowk[k]) != CC_READ)
          st_word(a.nodes + 4 * (pos[k] % a.n_nodes), 2 * (pos[k] / a.n_nodes + 1));
    }
  }
  install_values<L, K>(t, s, commit, a);
  order_point<STRICT>();
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (commit && s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), to_word(ts, ts));
  *hi = 0;
  *lo = ts;
  if (!active) return COMMIT;
  if (overflow) return TS_OVERFLOW;
  return lock_fail ? ABORT_LOCK : (valid_fail ? ABORT_VALID : COMMIT);
}

// ===========================================================================
// TicToc (paper Section 2 "Optimistic Concurrency Control"; Section 3.5
// "OCC"; word = lock bit, 15-bit delta, 48-bit WTS with RTS = WTS + delta,
// Table 2).  Layout: bit 63 lock, bits 62-48 delta, bits 47-0 WTS.
//   R1  write rows: try-lock with fetch_or (abort if held); read rows: load
//       the word (abort if locked).
//   R2  read values; draw a ticket (tie-breaker for equal commit
//       timestamps); commit_ts = max over write rows of RTS+1 and over read
//       rows of WTS (team maximum).
//   R3  every read row must still carry the observed WTS and be unlocked (so
//       the value read in R2 is that version's); if its RTS < commit_ts,
//       extend RTS to commit_ts by CAS (if the delta would not fit in 15
//       bits, WTS is raised instead -- only other readers of the old WTS are
//       affected, and they abort).
//   R4  store values, wait, publish word = {WTS = commit_ts, delta = 0}.
// Serial key (commit_ts, ticket).
// ===========================================================================
constexpr uint64_t TT_LOCK = 1ull << 63;
constexpr uint64_t TT_WTS_MASK = (1ull << 48) - 1ull;
constexpr uint64_t TT_DELTA_MAX = (1ull << 15) - 1ull;
__device__ __forceinline__ uint64_t tt_wts(uint64_t w) { return w & TT_WTS_MASK; }
__device__ __forceinline__ uint64_t tt_rts(uint64_t w) { return tt_wts(w) + ((w >> 48) & TT_DELTA_MAX); }

template <int L, int K, bool STRICT, bool LATCH>
__device__ __forceinline__ int tictoc_attempt(const Team<L> &t, Slots<K> &s, bool active, const RunArgs &a,
                                              bool precheck, uint64_t *hi, uint64_t *lo) {
  bool fail = false;
  uint32_t blk = ~0u;
  bool pre_fail = false;
  if (ballot(active && precheck)) {
    // R0 (as OCC's, by default from a transaction's second attempt on): load
    // every row's word and give up before locking if one is held; read-only
    // rows keep the word loaded here, exactly as R1 would load it
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (active && precheck && s.valid[k] && op_leader(s.rowk[k])) {
        const uint64_t o = ld_word(a.words + op_row(s.rowk[k]));
        s.v[k] = o;
        if ((o & TT_LOCK) && blk == ~0u) blk = op_row(s.rowk[k]);
        fail |= (o & TT_LOCK) != 0;
      }
    }
    order_point<STRICT>();
    pre_fail = t.any(fail);
  }
  const bool go = active && !pre_fail;
  // locks and loads all issued before any result is looked at (see OCC's R1)
  bool issued[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.got[k] = false;
    issued[k] = go && s.valid[k] && op_leader(s.rowk[k]) && (!precheck || op_written(s.rowk[k]));
    if (issued[k]) {
      uint64_t *w = a.words + op_row(s.rowk[k]);
      if (op_written(s.rowk[k])) s.v[k] = w_or<LATCH, STRICT>(a, w, TT_LOCK);
      else s.v[k] = ld_word(w);
    }
  }
  order_point<STRICT>();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!issued[k]) continue;
    const uint64_t o = s.v[k];
    if ((o & TT_LOCK) && blk == ~0u) blk = op_row(s.rowk[k]);
    if (op_written(s.rowk[k])) s.got[k] = !(o & TT_LOCK);
    fail |= (o & TT_LOCK) != 0;
  }
  s.block = blocking_row(t, blk);
  const bool lock_fail = t.any(fail);
  const bool alive = active && !lock_fail;
  if (active && lock_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
  }
  uint64_t cts = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (alive && s.valid[k]) {
      s.x[k] = ld_val(a.data + s.elem[k]);
      if (op_leader(s.rowk[k])) {
        const uint64_t c = op_written(s.rowk[k]) ? tt_rts(s.v[k]) + 1 : tt_wts(s.v[k]);
        cts = c > cts ? c : cts;
      }
    }
  }
  const uint64_t ticket = t.claim(&a.ctl->ticket, alive, 1) + 1;
  cts = t.max(cts);
  const bool overflow = alive && cts > TT_WTS_MASK - TT_DELTA_MAX;
  order_point<STRICT>();
  bool bad = overflow;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (alive && !overflow && s.valid[k] && op_leader(s.rowk[k]) && !op_written(s.rowk[k])) {
      // the value read in R2 belongs to the observed version only if the row
      // is still unlocked with the same WTS now (a writer installs values
      // while holding the lock, then publishes a new WTS)
      uint64_t *wp = a.words + op_row(s.rowk[k]);
      uint64_t w = ld_word(wp);
      bool done = false, b = false;
      for (int it = 0; it < CAS_RETRIES && !done && !b; ++it) {
        if (tt_wts(w) != tt_wts(s.v[k]) || (w & TT_LOCK)) {
          b = true;
        } else if (tt_rts(w) >= cts) {
          done = true;
        } else {
          uint64_t wts = tt_wts(w), delta = cts - wts;
          if (delta > TT_DELTA_MAX) {
            wts = cts - TT_DELTA_MAX;
            delta = TT_DELTA_MAX;
          }
          if (w_cas<LATCH, STRICT>(a, wp, &w, wts | (delta << 48))) done = true;
        }
      }
      bad |= b || !done;
    }
  }
  const bool valid_fail = t.any(bad);
  const bool commit = alive && !valid_fail;
  if (alive && valid_fail) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), s.v[k]);
  }
  install_values<L, K>(t, s, commit, a);
  order_point<STRICT>();
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (commit && s.got[k]) w_st<LATCH, STRICT>(a, a.words + op_row(s.rowk[k]), cts);
  *hi = cts;
  *lo = ticket;
  if (!active) return COMMIT;
  if (overflow && !lock_fail) return TS_OVERFLOW;
  return lock_fail ? ABORT_LOCK : (valid_fail ? ABORT_VALID : COMMIT);
}

}  // namespace cce
