// Internal layout shared by the host runtime (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cc.h"

namespace cce {

// ---- device operation descriptor (16 B) ------------------------------------
// rowk packs the global row id (row within its table + the table's first row
// in the shared row-id space) with the op kind and two flags computed at
// submission:
//   FOLLOWER  the op touches the same row as the previous op of its txn, so
//             the row's first op ("leader") does the concurrency control;
//   WRITTEN   some op of the row group writes the row.
// elem is the cell index in the value arena (table base + row*fields + field).
struct DevOp {
  uint32_t rowk;
  uint32_t elem;
  int64_t arg;
};
static_assert(sizeof(DevOp) == 16, "DevOp is 16 bytes");

constexpr uint32_t ROW_BITS = 28;
constexpr uint32_t ROW_MASK = (1u << ROW_BITS) - 1u;
constexpr uint32_t KIND_SHIFT = 28;
constexpr uint32_t FOLLOWER_BIT = 1u << 30;
constexpr uint32_t WRITTEN_BIT = 1u << 31;

struct DevTxn {
  uint32_t first;  // first op
  uint32_t n;      // op count
};

struct DevOutcome {  // same layout as cc_outcome
  uint32_t status;
  uint32_t attempts;
  uint64_t serial_hi;
  uint64_t serial_lo;
  int64_t commit_ns;
};
static_assert(sizeof(DevOutcome) == sizeof(cc_outcome), "outcome layout");

// ---- device control block, cleared by the init kernel ----------------------
enum DevStat {
  DS_COMMITTED = 0,
  DS_ATTEMPTS = 1,
  DS_ABORT_LOCK = 2,
  DS_ABORT_VALID = 3,
  DS_GAVE_UP = 4,
  DS_MAX_ATTEMPTS = 5,
  DS_TS_OVERFLOW = 6,
  DS_DEFERRED = 7,
  DS_T_USEFUL = 8,  // wall-clock ticks, summed over teams
  DS_T_ABORT = 9,
  DS_T_WAIT = 10,
  DS_ADMIT_WAITS = 11,  // serving: admissions deferred because the byte budget was full
  DS_R1 = 12,           // OCC, committed attempts: ticks in each round (lock / read+ticket /
  DS_R2 = 13,           //   validate+install / release)
  DS_R3 = 14,
  DS_R4 = 15,
  DS_INDEX_MISS = 16,   // keyed operations whose key no row holds
  DS_WD_WAITS = 17,     // 2PL wait-die: times a team kept its locks and waited
  DS_LATCH_STUCK = 18,  // CC_RUN_LATCH: latches not obtained within the spin limit (run invalid)
  DS_HOT_ACQ = 19,      // OCC: acquisitions of the batch's most written row's lock
  DS_HOT_FAILED = 20,   //   of which the attempt then aborted
  DS_HOT_HOLD = 21,     //   ticks the row was held, summed over acquisitions
  DS_BLOCKED_WAITS = 22,// CC_RUN_WAIT_BLOCKER: waits for a held row entered
  DS_VERSION_MISS = 23, // MVCC: old-version reads that found their version's slot reused (attempt aborted)
  DS_ENGINE_WAITS = 24, // OCC hot-row engine: times a team kept its locks and waited for an engine row
  DS_N = 25
};

struct Ctl {
  uint64_t queue;        // next transaction index to hand out
  uint64_t ticket;       // serial ticket / timestamp counter (last value drawn)
  uint64_t start_clock;  // device wall clock at CC initialisation
  uint64_t pending_n;    // length of the pending list built between passes
  uint64_t budget_reserved;  // serving: bytes ever reserved (a FIFO position counter)
  uint64_t budget_released;  // serving: bytes ever released
  uint64_t stats[DS_N];
  uint64_t stop;             // set by a team whose wait exceeded its limit (GaccO, GPUTx) or whose latch
                             // was stuck (CC_RUN_LATCH); every team then exits
};

// Kernel arguments for a transaction run.
// Rows a batch's submission singles out as hot (most writes first).
constexpr int HOT_MAX = 8;

struct RunArgs {
  const DevOp *ops;
  const DevTxn *txns;
  const uint32_t *list;  // transactions of this pass (nullptr: 0..n_txns-1)
  uint64_t n_txns;       // transactions in this pass
  int64_t *data;    // value arena
  uint64_t *words;  // one control word per global row
  uint64_t *aux;    // second word per row (MVCC version pointer)
  uint64_t *nodes;  // MVCC version arena: n_nodes slots of 4 words {tag, prev, writer ts | cell << 32, pre-image}
  uint64_t n_nodes;
  uint64_t *node_ring;  // MVCC: slots handed out so far (the arena is a ring; pos -> slot pos % n_nodes)
  DevOutcome *out;
  int64_t *reads;   // per op read value
  Ctl *ctl;
  uint64_t max_attempts;
  uint32_t backoff_ticks;  // wall-clock ticks
  uint32_t ns_per_tick_q16;  // wall-clock tick length in ns, 16.16 fixed point
  uint32_t has_slot;       // batch contains WRITE_SLOT ops
  uint32_t defer_after;    // attempts in this pass before deferring (0: never)
  uint32_t pass;           // 0 for the first pass (attempt counts start at 0)
  uint32_t n_from_ctl;     // take the pass's transaction count from ctl->pending_n
  const int64_t *arrival;  // serving: arrival time of each transaction, wall-clock ticks after start
  uint64_t budget_cap;     // serving: admission cap on reserved bytes (0: no cap)
  uint32_t bytes_per_op;   // serving: log / version bytes one operation reserves
  uint32_t eager_install;  // OCC: store values in the validation round (undo on abort)
  uint32_t pad4;
  uint32_t precheck;       // OCC, TicToc, TO, MVCC: load-only round before any lock: 0 never, 1 on retries, 2 always
  uint32_t wd_wait_limit;  // 2PL wait-die: waits of one attempt before it dies anyway
  uint32_t node_reuse;     // MVCC: 0 = a slot per op (op i keeps slot i, never reused); 1 = the ring protocol
  uint32_t *latch;         // CC_RUN_LATCH: one 32-bit latch per global row (else unused)
  // OCC: the batch's hottest written rows (most writes first), locked -- or,
  // for a read-only access, looked at -- in a round of their own once every
  // other row of the transaction is held (0 rows: one lock round)
  uint32_t n_late;
  uint32_t late[HOT_MAX];
  uint32_t hot0;           // the batch's most written row (~0u: none), for the hold statistics
  // OCC, TicToc (CC_RUN_WAIT_BLOCKER): in passes that defer, a team that failed
  // on a held row looks at that row's word every ~poll_ticks until it is free
  // or wait_max_ticks have passed, then retries after a random jitter below
  // jitter_ticks, instead of backing off
  uint32_t wait_blocker;
  uint32_t poll_ticks;
  uint32_t jitter_ticks;
  uint32_t pad7;
  uint64_t wait_max_ticks;
};

// A table's index on the device (index.hip): the table's keys sorted, with
// their rows, and a static 16-way search tree over them.  Level 0 is the
// sorted keys, padded with INT64_MAX to a multiple of 16; level l+1 holds the
// largest key of each 16-key node of level l, padded the same way; the top
// level is one node.
constexpr int INDEX_MAX_LEVELS = 8;
struct IndexDesc {
  const int64_t *keys;   // level 0
  const uint32_t *rows;  // row of each sorted key
  const int64_t *tree;   // levels 1..levels, level l at level_off[l]
  uint64_t n;            // keys (rows of the table)
  uint64_t level_off[INDEX_MAX_LEVELS + 1];
  uint64_t row_base;     // the table's first global row
  uint64_t elem_base;    // the table's first cell
  uint32_t n_fields;
  uint32_t levels;       // tree levels above level 0
};

// OCC hot-row engine (hot_engine.h): the batch's most written rows, held in
// one workgroup's LDS while the transactions that write them run there.
// Rows of at most ENG_FIELDS fields, ENG_VALS cells in all.
constexpr int ENG_MAX = 32;
constexpr int ENG_FIELDS = 64;
constexpr int ENG_VALS = 1024;
struct EngineDesc {           // one engine transaction: its id, first op and op count, and the
  uint32_t txn, first, n, emask;  // engine rows it touches (bit k: engine row k)
};
struct EngineArgs {
  const EngineDesc *desc;     // the engine's transactions, in batch order
  uint64_t n_txns;
  uint32_t n_rows;            // engine rows (0: no engine)
  uint32_t n_vals;            // their cells
  uint32_t row[ENG_MAX];      // global row of engine row i
  uint32_t elem0[ENG_MAX];    // its first cell in the value arena
  uint32_t off[ENG_MAX + 1];  // its first cell in LDS; off[n_rows] = n_vals
  uint32_t pad[2];
};

// Per-op metadata of a keyed batch: bit 31 keyed, bits 16-23 table, 0-7 field.
constexpr uint32_t META_KEYED = 1u << 31;

// Resolve the keys of a keyed batch: patch each keyed op's row and cell in
// `ops`, record its row (within its table) in rows_out, count misses in
// ctl->stats[DS_INDEX_MISS].  tree = false: binary search of the sorted keys;
// true: descent of the 16-way tree.  One lane per op either way.
hipError_t launch_index_lookup(hipStream_t s, bool tree, const int64_t *op_keys, const uint32_t *meta, DevOp *ops,
                               uint32_t *rows_out, uint64_t n_ops, const IndexDesc *idx, Ctl *ctl);

// Kernel arguments for a GaccO execution (gacco_exec.hip).
struct GaccoArgs {
  const DevOp *ops;
  const DevTxn *txns;
  uint64_t n_txns;
  const uint32_t *rank;  // per row-group leader: its position in the sorted access table
  int64_t *data;
  uint64_t *words;       // per row: the position whose turn it is
  DevOutcome *out;
  int64_t *reads;
  Ctl *ctl;
  uint64_t wait_limit_ticks;  // a team waiting longer than this without progress stops the run
  uint32_t poll_ticks;        // sleep per access queued ahead of the team on a row, wall-clock ticks
  uint32_t ns_per_tick_q16;
  uint32_t has_slot;
  uint32_t shared;            // CC_RUN_SHARED_READS: counters instead of turns (see gacco_prepare)
};

// GaccO preprocessing (gacco.hip): clears ctl->stop, then builds the access
// table, sorts it stably by row (radix sort) and writes the lock table (turn
// counters in `words`, per-leader ranks).  `scratch` holds
// gacco_scratch_words(n_ops) 32-bit words.
uint64_t gacco_scratch_words(uint64_t n_ops);
// Stable LSD radix sort (8-bit digits) of n (key, value) pairs on their low
// `bits` key bits.  keys/vals are sorted through `scratch`
// (radix_sort_scratch_words(n) words); *keys_out / *vals_out point at the
// result (the input arrays or the first 2n words of scratch).
uint64_t radix_sort_scratch_words(uint64_t n);
hipError_t radix_sort_pairs(hipStream_t s, uint32_t *keys, uint32_t *vals, uint64_t n, int bits, uint32_t *scratch,
                            uint32_t **keys_out, uint32_t **vals_out);
// Modes:
//  PREP_TURNS   each accessed row's word is the sorted position of its first
//               access, and a leader's rank is its own sorted position (the
//               turn it waits for);
//  PREP_SHARED  the words hold (accesses done, writes done) counters and a
//               leader's rank is its threshold: accesses before it in its row
//               for a write, writes before it for a read (reads between two
//               writes share the row);
//  PREP_LOCAL   every accessed row's word is 0 and a leader's rank is its
//               place in its row's list (GPUTx's packed rank state).
enum PrepMode { PREP_TURNS = 0, PREP_SHARED = 1, PREP_LOCAL = 2 };
hipError_t gacco_prepare(hipStream_t s, const DevOp *ops, uint64_t n_ops, uint32_t sentinel, uint64_t *words,
                         uint32_t *rank, uint32_t *scratch, Ctl *ctl, int mode);
// GaccO execution; hipErrorInvalidValue for an unsupported (lanes, ops per txn).
hipError_t launch_gacco(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, bool strict,
                        const GaccoArgs &a, int n_cu, int *grid_used);

// Kernel arguments for the GPUTx passes (gputx.hip).
struct GputxArgs {
  const DevOp *ops;
  const DevTxn *txns;
  uint64_t n_txns;
  const uint32_t *rank;       // per row-group leader: its place in its row's list (the turn it waits for)
  uint64_t *words;            // per row: the turn
  uint64_t *kstate;           // per row: (largest rank + 1 of its accessors so far) << 32 | (last writer's rank + 1)
  uint32_t *txn_rank;         // rank pass output: per transaction
  const uint32_t *order;      // execution: transaction at each sorted position
  const uint32_t *order_rank; // execution: its rank
  const uint32_t *kstart;     // execution: first sorted position of each rank
  int64_t *data;
  DevOutcome *out;
  int64_t *reads;
  Ctl *ctl;
  uint64_t wait_limit_ticks;
  uint32_t poll_ticks;
  uint32_t ns_per_tick_q16;
  uint32_t has_slot;
  uint32_t packed;            // rank pass: turn and rank state share the row's word (see gputx.hip)
};
hipError_t launch_gputx_pass(hipStream_t s, bool exec, int lanes, int max_ops, int waves_per_wg, int grid,
                             bool strict, const GputxArgs &a, int n_cu, int *grid_used);
hipError_t gputx_init_state(hipStream_t s, uint64_t *kstate, uint64_t n_rows, uint32_t *iota, uint64_t n_txns);
hipError_t gputx_reset(hipStream_t s, Ctl *ctl);
hipError_t gputx_kstart(hipStream_t s, const uint32_t *rank_sorted, uint64_t n, uint32_t *kstart);

// Device-side ingest of a batch already in device memory (ingest.hip).
struct IngestTable {
  uint64_t n_rows;
  uint64_t row_base;   // first global row
  uint64_t elem_base;  // first cell
  uint32_t n_fields;
  uint32_t indexed;    // keyed batches: the table has an index (its ops name rows by key)
};
// reduced results in IngestArgs::out
enum IngestOut { INGEST_ERR = 0, INGEST_MAX_OPS = 1, INGEST_HAS_SLOT = 2, INGEST_UNORDERED = 3, INGEST_KEYED = 4,
                 INGEST_N = 5 };
// what failed (bits 4-15 of the error word); the host turns it into a message
enum IngestMsg {
  INGEST_MSG_RESERVED = 1,
  INGEST_MSG_TOO_MANY,
  INGEST_MSG_OP_RANGE,
  INGEST_MSG_SHARED,
  INGEST_MSG_TABLE,
  INGEST_MSG_KEYED_ROW,
  INGEST_MSG_ROW_FIELD,
  INGEST_MSG_KIND,
  INGEST_MSG_SLOT_SRC,
  INGEST_MSG_DUP_FIELD,
  INGEST_MSG_DUP_ROW
};
struct IngestArgs {
  const cc_txn *txns;     // caller's device arrays
  const cc_op *ops;
  const int64_t *op_keys; // keyed batches (else nullptr)
  uint64_t n_txns, n_ops;
  IngestTable tab[CC_MAX_TABLES];
  uint32_t n_tables;
  uint32_t pad;
  DevOp *dops;            // packed descriptors (the batch's own buffers)
  DevTxn *dtx;
  uint32_t *owner;        // n_ops scratch words: lowest transaction naming each op
  uint32_t *meta;         // keyed batches: per-op keyed flag, table, field (else nullptr)
  uint32_t *rows0;        // keyed batches: per-op row as submitted
  uint64_t *out;          // INGEST_N words
};
// Resets out, then validates and packs; the host reads `out` afterwards.
hipError_t launch_ingest(hipStream_t s, const IngestArgs &a);

// Host-side launchers (kernels.hip).
hipError_t launch_init(hipStream_t s, uint64_t *words, uint64_t n_words, uint64_t *aux, uint64_t n_aux,
                       DevOutcome *out, uint64_t n_out, Ctl *ctl, uint64_t ticket_start);

// Between passes: list the transactions neither committed nor given up, and
// reset the claim counter.  ctl->pending_n receives the count.
hipError_t launch_compact(hipStream_t s, const DevOutcome *out, uint64_t n_txns, uint64_t max_attempts,
                          uint32_t *list, Ctl *ctl);

// Runs one plain batch: returns hipErrorInvalidValue for an unsupported
// (lanes, ops-per-lane) combination.
hipError_t launch_txn(hipStream_t s, int scheme, int lanes, int max_ops, int waves_per_wg, int grid,
                      bool strict, bool latch, const RunArgs &a, int n_cu, int *grid_used);

// The OCC hot-row engine over e.list (txn_occ.hip): one workgroup of `waves`
// wavefronts (0: the largest size the (lanes, ops-per-lane) variant allows);
// hipErrorInvalidValue for a combination it has no variant for (more than 4
// ops per lane).
hipError_t launch_engine_occ(hipStream_t s, int lanes, int max_ops, int waves, bool strict, const RunArgs &a,
                             const EngineArgs &e, int *threads_used);

// Per-scheme launchers (txn_<scheme>.hip).
#define CCE_DECLARE_LAUNCH(NAME)                                                                    \
  hipError_t NAME(hipStream_t s, int lanes, int max_ops, int waves_per_wg, int grid, bool strict, bool latch, \
                  const RunArgs &a, int n_cu, int *grid_used);
CCE_DECLARE_LAUNCH(launch_txn_occ)
CCE_DECLARE_LAUNCH(launch_txn_2pl)
CCE_DECLARE_LAUNCH(launch_txn_to)
CCE_DECLARE_LAUNCH(launch_txn_mvcc)
CCE_DECLARE_LAUNCH(launch_txn_tictoc)
CCE_DECLARE_LAUNCH(launch_txn_2plwd)
#undef CCE_DECLARE_LAUNCH

// The allocation-free run's device buffers (static_run.hip): one file-scope
// array per device, carved into the regions below.  Sizes follow
// CC_STATIC_MAX_TXNS and CC_STATIC_MAX_OPS (cc.h).
constexpr uint64_t STATIC_OFF_OPS = 0;
constexpr uint64_t STATIC_OFF_TXNS = STATIC_OFF_OPS + (uint64_t)CC_STATIC_MAX_OPS * sizeof(DevOp);
constexpr uint64_t STATIC_OFF_LIST = STATIC_OFF_TXNS + (uint64_t)CC_STATIC_MAX_TXNS * sizeof(DevTxn);
constexpr uint64_t STATIC_OFF_OWNER = STATIC_OFF_LIST + (uint64_t)CC_STATIC_MAX_TXNS * sizeof(uint32_t);
constexpr uint64_t STATIC_OFF_INGEST = STATIC_OFF_OWNER + (uint64_t)CC_STATIC_MAX_OPS * sizeof(uint32_t);
constexpr uint64_t STATIC_SCRATCH_BYTES = STATIC_OFF_INGEST + 256;
static_assert(STATIC_OFF_TXNS % 256 == 0 && STATIC_OFF_LIST % 256 == 0 && STATIC_OFF_OWNER % 256 == 0 &&
                  STATIC_OFF_INGEST % 256 == 0 && INGEST_N * sizeof(uint64_t) <= 256,
              "static scratch regions are 256-byte aligned");
// Device address of `device`'s array; `device` must be current.  Resolved
// with hipGetSymbolAddress on a device's first call, then kept.
constexpr int STATIC_MAX_DEVICES = 64;
hipError_t static_scratch_address(int device, void **ptr);
// Clears n int64 words with a fill kernel.
hipError_t launch_fill_zero(hipStream_t s, int64_t *p, uint64_t n);

// Memory micro-benchmarks (roofline.hip); see cc_probe in cc.h.
hipError_t run_probe(hipStream_t s, int kind, uint64_t footprint_bytes, uint64_t n_ops, int peer,
                     const uint64_t *host_idx, double *ms_out, uint64_t *err_out, int n_cu);

}  // namespace cce
