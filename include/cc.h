/*
 * cc.h -- C-ABI of the MI355X (gfx950) batch transaction engine.
 *
 * The engine executes a batch of read / read-modify-write transactions
 * concurrently against tables resident in device memory (HBM), under one of
 * seven concurrency-control schemes, and reports per transaction a serial key
 * that orders the committed transactions into an equivalent serial execution.
 *
 * Problem statement followed (paper Section 4.1, "Constraints" and
 * "Experimental Procedure"): tables and transactions are in device memory
 * before execution; transactions only read and write existing tuples (no
 * insert or delete); every transaction's read and write set is fixed before
 * execution; each transaction is restarted after a conflict until it
 * commits; all schemes guarantee serializable isolation (Section 3, "CC
 * Schemes Migration and Implementation").  The batch execution model with one
 * worker per transaction is Section 3.3 ("An Overview").
 *
 * Conventions for every call:
 *   - Return value: CC_OK (0) or a negative cc_status; no call throws, aborts
 *     or exits.  cc_strerror() names a status, cc_last_error() gives the
 *     message of the last failing call on a context.
 *   - Pointers named *_host are host memory; a flag argument `on_device`
 *     switches an array argument to a device pointer (for example a
 *     torch.Tensor.data_ptr() on the context's device).  The caller owns every
 *     array it passes; the engine copies inputs before the call returns and
 *     never keeps a caller pointer.
 *   - A context is used by one host thread at a time.  Work is issued on the
 *     stream given at cc_init (if NULL, a stream the context creates with the
 *     default priority); calls that return results synchronise that stream.
 *   - All table values are int64; arithmetic wraps in two's complement.
 */
#ifndef CC_H_
#define CC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cc_ctx cc_ctx;
typedef int32_t cc_status;

/* Status codes. */
#define CC_OK 0
#define CC_E_INVAL (-1)       /* malformed argument, unknown scheme/kind, bad run parameter */
#define CC_E_RANGE (-2)       /* table, row or field out of range; size limit exceeded */
#define CC_E_DUPROW (-3)      /* a (table,row) repeats non-adjacently, or a (table,row,field) repeats, within a txn */
#define CC_E_NOMEM (-4)       /* device or host allocation failed */
#define CC_E_TS_OVERFLOW (-5) /* a scheme's timestamp field would overflow; the run is invalid */
#define CC_E_LIVELOCK (-6)    /* transactions still pending after max_attempts / max_epochs */
#define CC_E_HIP (-7)         /* HIP runtime error (message in cc_last_error) */
#define CC_E_NODEV (-8)       /* no usable gfx950 device */
#define CC_E_STATE (-9)       /* call out of order (e.g. cc_create_table after the first cc_load) */
#define CC_E_NOBATCH (-10)    /* unknown batch id */

/* Concurrency-control schemes (paper Section 2 and Table 2; Section 3.5). */
enum cc_scheme {
  CC_OCC = 0,    /* Silo-style optimistic CC: lock bit + 63-bit TID per row */
  CC_2PL_NW = 1, /* two-phase locking, no-wait */
  CC_TO = 2,     /* basic timestamp ordering: commit bit + 31-bit RTS + 31-bit WTS */
  CC_MVCC = 3,   /* multi-version timestamp ordering (TO word + version pointer) */
  CC_TICTOC = 4, /* TicToc: lock bit + 15-bit delta + 48-bit WTS */
  CC_GACCO = 5,  /* GaccO, conflict-graph ordering (Section 2 and Section 3, "Conflict Graph
                    Ordering"): preprocessing sorts every row's accesses by transaction id into
                    a lock table; each row is then handed to its accessors in that order, reads
                    and writes alike.  Deterministic, no aborts.  Needs each transaction's ops
                    after the previous transaction's (first_op nondecreasing) and
                    CC_MODE_PLAIN; accepts only CC_RUN_STRICT_FENCES, CC_RUN_INDEX_TREE and
                    CC_RUN_SHARED_READS. */
  CC_2PL_WD = 6, /* two-phase locking, wait-die (Section 2 "Two-Phase Locking", Section 3.5): a
                    transaction older than the exclusive holder of a lock it needs keeps its
                    locks and waits (a state of its team, at most 64 times per attempt); any
                    other conflict aborts it.  Age = index in the batch.  Lock word as 2PL. */
  CC_GPUTX = 7   /* GPUTx, conflict-graph ordering by K-sets (Section 2 and Section 3, "Conflict
                    Graph Ordering"): a transaction's rank is its level in the DAG of
                    conflicts ordered by transaction id; the transactions of one rank run
                    together without concurrency control, rank after rank.  Deterministic, no
                    aborts.  Same batch and run rules as CC_GACCO. */
};
#define CC_N_SCHEMES 8

/*
 * Operation kinds.  An operation touches one field of one row.  Its read
 * value (reported by cc_fetch_outcomes) is always the field's value before
 * the operation (the pre-image).
 *   CC_READ       no change.
 *   CC_ADD        value + arg.
 *   CC_COND_ADD   v = value + arg; if v < CC_COND_LO then v += CC_COND_HI
 *                 (the stock-replenishing update of TPC-C NewOrder, a
 *                 workload the paper evaluates in Section 4.1).
 *   CC_WRITE_SLOT value := read[src] * mul + add, where read[src] is the read
 *                 value of operation `src` (an index within the same
 *                 transaction, smaller than this operation's index).  arg
 *                 packs src in bits 0-7, mul as a signed 24-bit integer in
 *                 bits 8-31 and add as a signed 32-bit integer in bits 32-63.
 * Within a transaction all operations on one (table,row) must be adjacent and
 * a (table,row,field) may appear at most once (else CC_E_DUPROW); the row
 * group is one row access for concurrency control.
 */
enum cc_op_kind { CC_READ = 0, CC_ADD = 1, CC_COND_ADD = 2, CC_WRITE_SLOT = 3 };
#define CC_COND_LO 10
#define CC_COND_HI 91

/* Limits. */
#define CC_MAX_OPS_PER_TXN 256
#define CC_MAX_TABLES 16
#define CC_MAX_TOTAL_ROWS (1ull << 28)   /* summed over all tables */
#define CC_MAX_TOTAL_CELLS (1ull << 32)  /* summed rows x fields over all tables */
#define CC_STATIC_MAX_TXNS (1u << 18)     /* cc_run_static: transactions per call */
#define CC_STATIC_MAX_OPS (1u << 20)      /* cc_run_static: ops per call */

typedef struct {
  uint32_t row;   /* row index within the table */
  uint16_t table; /* table id from cc_create_table */
  uint8_t field;  /* field index within the row */
  uint8_t kind;   /* enum cc_op_kind */
  int64_t arg;
} cc_op; /* 16 bytes */

typedef struct {
  uint64_t first_op; /* index of the transaction's first op in the ops array */
  uint32_t n_ops;    /* number of ops, 0..CC_MAX_OPS_PER_TXN */
  uint32_t reserved; /* must be 0 */
} cc_txn; /* 16 bytes */

enum cc_txn_status { CC_PENDING = 0, CC_COMMITTED = 1 };

/*
 * Per-transaction outcome.  Sorting committed transactions by
 * (serial_hi, serial_lo) gives a serial order equivalent to the run:
 *   OCC, 2PL (both forms):  (0, ticket)  -- ticket drawn from one device
 *                              counter while the transaction holds all its
 *                              write locks;
 *   TO, MVCC:  (0, ts)      -- the timestamp of the committing attempt;
 *   TicToc:    (commit_ts, ticket);
 *   GaccO:     (0, transaction index) -- the scheme's order is the id order;
 *   GPUTx:     (rank, transaction index) -- K-set, then id.
 * attempts counts executions of the transaction, so attempts-1 are aborts
 * (the paper's abort rate is aborts / committed, Section 4.1 "Metric
 * Selection").  commit_ns is the device wall-clock time of the commit,
 * relative to the start of the run (CC initialisation).
 */
typedef struct {
  uint32_t status;
  uint32_t attempts;
  uint64_t serial_hi;
  uint64_t serial_lo;
  int64_t commit_ns;
} cc_outcome; /* 32 bytes */

typedef struct {
  int32_t device;  /* HIP device ordinal */
  uint32_t flags;  /* must be 0 */
  void *stream;    /* hipStream_t to issue work on (e.g. a torch stream); NULL: the context creates a
                      stream of its own with the default priority (so that its runs can be captured) */
} cc_config;

/*
 * Run modes.
 *   CC_MODE_PLAIN  the paper's procedure (Section 4.1, "Experimental
 *                  Procedure"): each transaction is retried in-kernel until it
 *                  commits; after defer_after failed attempts it moves to a
 *                  later pass with 8x fewer workgroups.
 *   CC_MODE_EPOCH  batching: in each epoch every pending transaction gets
 *                  defer_after (default 1) attempts on a persistent grid; the
 *                  aborted ones wait for the next epoch.  Four epochs are
 *                  captured as one hipGraph and replayed until nothing is
 *                  pending (max_epochs bounds the total: CC_E_LIVELOCK).
 *   CC_MODE_SERVE  continuous batching over a stream: transactions are taken
 *                  in arrival order (cc_set_arrivals) by a persistent grid,
 *                  each starts no earlier than its arrival time on the device
 *                  clock and only once CC_SERVE_BYTES_PER_OP x its op count
 *                  fits in the hbm_cap_bytes budget of uncommitted work; it
 *                  releases the bytes when it commits; aborts retry after
 *                  back-off while later arrivals proceed.  Latency statistics
 *                  are commit time minus arrival time.  Under CC_MVCC the
 *                  cap also sizes the version arena (hbm_cap_bytes / 32
 *                  slots, reused as a ring; CC_STAT_VERSION_SLOTS), so the
 *                  device memory that old versions take is bounded by the cap
 *                  however long the stream; a reader whose version's slot was
 *                  reused aborts and retries with a newer timestamp.
 */
enum cc_mode { CC_MODE_PLAIN = 0, CC_MODE_EPOCH = 1, CC_MODE_SERVE = 2 };
#define CC_SERVE_BYTES_PER_OP 32 /* read value + new value + undo / version record, 8 B each + 8 B index */

/* Run flags. */
#define CC_RUN_STRICT_FENCES 0x1u /* agent-scope acquire/release fences (cache invalidate/write-back) at
                                     every ordering point instead of wait-for-completion only */
#define CC_RUN_WAIT_UNLOCK 0x4u   /* reserved; always rejected with CC_E_INVAL (a retry-when-free policy
                                     whose teams of one wavefront could retry in lockstep and livelock
                                     in the final single-wavefront pass; the code path is removed) */
#define CC_RUN_PRECHECK 0x8u      /* OCC, TicToc, TO and MVCC: an extra first round loads every row's word and aborts before
                                     taking any lock if one is held -- on every attempt.  By default it
                                     runs from a transaction's second attempt on (a failure is the
                                     sign of contention) when the batch's most written row takes writes
                                     from at least 2% of its transactions, and never below that, where
                                     the extra round costs more than it saves.  CC_E_INVAL for another
                                     scheme, or together with CC_RUN_NO_PRECHECK */
#define CC_RUN_NO_PRECHECK 0x10u  /* OCC, TicToc, TO and MVCC: never run the pre-check round (CC_E_INVAL for
                                     another scheme) */
#define CC_RUN_LATCH 0x40u        /* latch variants of the non-deterministic schemes (paper Section 4.2,
                                     Exp-7): a 32-bit latch per row guards its control word, and every
                                     update of the word is a critical section [latch, load, store,
                                     unlatch] instead of one 64-bit atomic.  Not for CC_GACCO or CC_GPUTX.
                                     A latch not obtained within 2^22 tries fails the run: every team
                                     stops, cc_run returns CC_E_LIVELOCK, and the table contents are
                                     undefined (reload them before the next run) */
#define CC_RUN_SHARED_READS 0x80u /* CC_GACCO: reads of a row between two of its writes run together (a
                                     write still waits for every earlier access, a read for every
                                     earlier write); the paper's GaccO queues reads like writes */
#define CC_RUN_INDEX_TREE 0x20u   /* keyed batches: look keys up by descending the index's 16-way tree
                                     (one 128-byte node per level) instead of by binary search of the
                                     sorted keys */
#define CC_RUN_HOT_LAST 0x100u    /* OCC: lock the batch's hottest rows (found at submission: at most 8, each
                                     written at least a quarter as often as the hottest) in a round of their
                                     own, after every other row of the transaction is held, so that a hot
                                     row is held only for the commit rounds and never by an attempt that
                                     fails on another row's lock.  Off by default: the extra round lengthens
                                     every attempt and the read rows' validation window, which costs more
                                     than the shorter holds save.  Not applied with one lane per
                                     transaction or 16 ops per lane. */
#define CC_RUN_NO_HOT_LAST 0x200u /* OCC: one lock round for every row, the default (CC_E_INVAL with
                                     CC_RUN_HOT_LAST) */
#define CC_RUN_WAIT_BLOCKER 0x400u /* OCC and TicToc (CC_E_INVAL for another scheme): after an attempt that
                                     failed on a row another transaction held, wait until that row is free
                                     -- its word looked at every ~2 back-off bases, at most 256 bases --
                                     then retry after a random jitter below 2 bases, instead of backing off.
                                     Only in passes that defer (CC_MODE_PLAIN's passes before the last,
                                     CC_MODE_SERVE); the final pass, which never defers, keeps the
                                     randomised back-off, so two transactions that block each other cannot
                                     retry in lockstep forever there */
#define CC_RUN_HOT_ENGINE 0x800u  /* OCC, CC_MODE_PLAIN (CC_E_INVAL otherwise, and with CC_RUN_LATCH): run
                                     the transactions that write one of the batch's most written rows
                                     first, in one workgroup that holds those rows in LDS (hot-row engine:
                                     up to 32 rows written at least max(2, n_txns / 4096) times, of at most
                                     64 fields, found at submission; CC_STAT_ENGINE_*).  There an engine
                                     row takes a reader-writer lock in LDS -- shared to read, exclusive to
                                     write -- and a transaction that finds it taken gives back what it holds
                                     and waits until it is free; the other rows follow OCC (lock written
                                     rows, validate read rows) and the ticket comes from an LDS counter.  The rest of the
                                     batch then runs as usual, with the engine rows only read.  Paper
                                     Section 2 "Optimistic Concurrency Control" and Section 3.5 "OCC", with
                                     hot rows locked pessimistically.  On by default for an OCC batch whose
                                     most written row is written by at least a tenth of its transactions,
                                     whose transactions have at most 32 ops, and whose rows left out of the
                                     engine are written at most a quarter as often as the most written one
                                     (elsewhere one workgroup carrying the hot rows' share loses to the
                                     whole GPU).  The engine runs one
                                     transaction per wavefront (64 lanes) and as many wavefronts as fit,
                                     unless lanes_per_txn / waves_per_wg are set; it needs at most 4 ops per
                                     lane (CC_E_INVAL at cc_run when forced without) and a batch submitted by
                                     row (the keyed path finds rows only at the run). */
#define CC_RUN_NO_HOT_ENGINE 0x1000u /* OCC: no hot-row engine (CC_E_INVAL with CC_RUN_HOT_ENGINE) */
#define CC_RUN_EAGER_INSTALL 0x2u /* OCC only (CC_E_INVAL for another scheme): store new values in the
                                     validation round (undo on abort) instead of after validation
                                     succeeds; measured ~3% slower on the key-value workload, kept for
                                     comparison */

typedef struct {
  uint32_t lanes_per_txn; /* lanes cooperating on one transaction: 1, 4, 16, 64; 0 = chosen by contention
                             (see below) */
  uint32_t waves_per_wg;  /* 64-lane wavefronts per workgroup, 1..16; 0 = chosen by contention */
  uint32_t grid;          /* workgroups of the first pass; 0 = one per compute unit
                             Defaults by contention, from the share h of transactions that write the
                             batch's most written row (counted at submission): below 0.1% (no hot row)
                             4 lanes per transaction and 4 wavefronts per workgroup when the longest
                             transaction has at most 64 ops, so that 4096 transactions are in flight;
                             otherwise one wavefront per workgroup and the smallest lane count
                             >= the longest transaction, which keeps fewer transactions in flight. */
  uint32_t mode;          /* enum cc_mode */
  uint64_t max_attempts;  /* give up (CC_E_LIVELOCK) after this many attempts of one txn; 0 = 1<<24 */
  uint32_t max_epochs;    /* CC_MODE_EPOCH: epochs before CC_E_LIVELOCK; 0 = 1<<20 */
  uint32_t flags;         /* CC_RUN_* */
  uint32_t backoff_ns;    /* base of the randomised exponential back-off after an abort; 0 = 200 ns */
  uint32_t defer_after;   /* CC_MODE_PLAIN: attempts of a transaction within one pass before it is deferred
                             to the next pass, which runs 8x fewer workgroups (the last pass runs one
                             wavefront and never defers); 0 = 16.  CC_MODE_EPOCH: attempts per epoch;
                             0 = 1 */
  uint64_t ts_start;      /* first value of the run's ticket / timestamp counter (0 for normal runs; a
                             large value forces the 31-bit TO/MVCC timestamp-overflow path) */
  uint64_t hbm_cap_bytes; /* CC_MODE_SERVE: admission budget for uncommitted work and, under CC_MVCC, the
                             version arena's size; 0 = no cap (one version slot per op of the stream) */
  uint64_t wait_limit_us; /* CC_GACCO, CC_GPUTX: a team that sees no progress on its waits for this long
                             stops every team and the run fails with CC_E_LIVELOCK; 0 = 4 s.  It cannot
                             trigger while the lock table is consistent (the smallest unfinished
                             transaction can always proceed); a tiny value exercises the stop path.
                             Nonzero for another scheme: CC_E_INVAL */
} cc_run_params;

/* Counters reported by cc_stats (index: meaning). */
enum cc_stat {
  CC_STAT_COMMITTED = 0,   /* committed transactions */
  CC_STAT_ATTEMPTS = 1,    /* transaction executions (commits + aborts) */
  CC_STAT_ABORT_LOCK = 2,  /* aborts: a lock / word was held by another transaction */
  CC_STAT_ABORT_VALID = 3, /* aborts: a read was invalidated, or a timestamp rule failed */
  CC_STAT_KERNEL_NS = 4,   /* execution time of the transaction kernel(s), HIP events */
  CC_STAT_RUN_NS = 5,      /* CC initialisation + execution (the paper's measured window) */
  CC_STAT_TICKETS = 6,     /* serial tickets / timestamps drawn */
  CC_STAT_MAX_ATTEMPTS = 7,/* largest attempts of one transaction */
  CC_STAT_LAT_P50_NS = 8,  /* commit latency percentiles over the batch (commit_ns) */
  CC_STAT_LAT_P99_NS = 9,
  CC_STAT_EPOCHS = 10,     /* epochs run (CC_MODE_EPOCH) */
  CC_STAT_PASSES = 11,     /* kernel passes run (CC_MODE_PLAIN) */
  CC_STAT_DEFERRED = 12,   /* transactions deferred to a later pass */
  CC_STAT_GRID = 13,       /* workgroups of the first pass */
  CC_STAT_T_USEFUL_NS = 14,/* summed over transactions: time in attempts that committed */
  CC_STAT_T_ABORT_NS = 15, /* summed over transactions: time in attempts that aborted */
  CC_STAT_T_WAIT_NS = 16,  /* summed over transactions: back-off time between attempts */
  CC_STAT_GAVE_UP = 17,    /* transactions left pending (attempt limit or timestamp overflow) */
  CC_STAT_ADMIT_WAITS = 18,/* CC_MODE_SERVE: admissions postponed because the byte budget was full */
  CC_STAT_OCC_R1_NS = 19,  /* OCC, summed over committed attempts: time in round 1 (locks, read words), */
  CC_STAT_OCC_R2_NS = 20,  /*   round 2 (values + ticket), round 3 (validation + install) and round 4 */
  CC_STAT_OCC_R3_NS = 21,  /*   (release) */
  CC_STAT_OCC_R4_NS = 22,
  CC_STAT_PREP_NS = 23,    /* GaccO: preprocessing (access table, radix sort, lock table), HIP events;
                              part of CC_STAT_RUN_NS */
  CC_STAT_INDEX_NS = 24,   /* keyed batches: the index lookups, HIP events; part of CC_STAT_RUN_NS */
  CC_STAT_WD_WAITS = 25,   /* CC_2PL_WD: times a transaction kept its locks and waited */
  CC_STAT_KSETS = 26,      /* CC_GPUTX: K-sets (largest rank + 1) */
  CC_STAT_PACKED_STATE = 27, /* CC_GPUTX: 1 if the rank pass kept each row's rank state in its turn word
                                (fewer than 2^20 transactions and 2^24 operations), else 0 */
  CC_STAT_HOT_ACQ = 28,    /* OCC: acquisitions of the lock of the batch's most written row */
  CC_STAT_HOT_FAILED = 29, /* OCC: of those, acquisitions whose attempt aborted (a failed hold) */
  CC_STAT_HOT_HOLD_NS = 30,/* OCC: time that row's lock was held, summed over acquisitions (the rest of
                              CC_STAT_KERNEL_NS it was free) */
  CC_STAT_HOT_WRITES = 31, /* writes to the batch's most written row (counted at submission) */
  CC_STAT_BLOCKED_WAITS = 32, /* CC_RUN_WAIT_BLOCKER: waits for a held row that failed attempts entered */
  CC_STAT_VERSION_SLOTS = 33, /* CC_MVCC: slots of the version arena (32 bytes each): one per op of the
                                 batch, or hbm_cap_bytes / 32 in CC_MODE_SERVE with a cap; at least 1024.
                                 With at least one slot per op, op i keeps slot i and no slot is
                                 reused; with fewer, the arena is a ring */
  CC_STAT_VERSION_MISSES = 34,/* CC_MVCC: old-version reads whose version's slot the ring had reused
                                 (the attempt aborted and retried with a newer timestamp) */
  CC_STAT_ENGINE_TXNS = 35,   /* hot-row engine (CC_RUN_HOT_ENGINE, or by default): transactions it ran
                                 (0: no engine) */
  CC_STAT_ENGINE_ROWS = 36,   /* hot-row engine: rows it held in LDS */
  CC_STAT_ENGINE_NS = 37,     /* hot-row engine: its kernel time (part of CC_STAT_KERNEL_NS) */
  CC_STAT_ENGINE_WAITS = 38,  /* hot-row engine: times a transaction found an engine row taken, gave back
                                 every row it held and waited for that row */
  CC_N_STATS = 40
};

/* Library version and self-description (no device work). */
const char *cc_version(void);
const char *cc_strerror(cc_status status);
const char *cc_last_error(const cc_ctx *ctx);

/*
 * Create a context on cfg->device (which must be a gfx950 GPU) issuing work
 * on cfg->stream (cfg NULL: device 0, own stream).  The context holds the
 * device state of one database (paper Section 3.3, "An Overview": tables,
 * control words and batches live in device memory, and the host only
 * launches work): its control block is allocated here.  *out receives the
 * context, or NULL on error.  Errors: CC_E_INVAL (out NULL, flags not 0),
 * CC_E_NODEV (no device, ordinal out of range, not gfx950), CC_E_NOMEM,
 * CC_E_HIP; cc_last_error(NULL) gives the message.
 */
cc_status cc_init(cc_ctx **out, const cc_config *cfg);

/*
 * Wait for the context's stream, then free every device and host resource
 * of the context (tables, indexes, batches, the stream it created).  The
 * caller's stream and buffers are not touched.  NULL is accepted.
 */
cc_status cc_destroy(cc_ctx *ctx);

/*
 * Declare a table of n_rows x n_fields int64 values (row store, paper
 * Section 3.4 "DBMS Building Blocks": a table is an array of tuples of fixed
 * size; all tables are laid out consecutively and share one row-id space).
 * Tables must be declared before the first cc_load; *table_id receives
 * 0, 1, 2, ... in declaration order.
 */
cc_status cc_create_table(cc_ctx *ctx, uint64_t n_rows, uint32_t n_fields, uint32_t *table_id);

/*
 * Copy n_rows x n_fields values (row-major) into a table: the data is
 * resident in device memory before any transaction runs (paper Section 4.1,
 * "Constraints").  n_rows must equal the table's row count.  rows is a host
 * pointer, or a device pointer when rows_on_device is non-zero
 * (device-to-device copy, e.g. a pristine copy kept in a torch tensor); the
 * caller keeps ownership and the call returns after the copy.  The first
 * cc_load lays out and allocates every declared table (one value arena, one
 * control word per row, Section 3.4) and freezes the set of tables.  Errors:
 * CC_E_INVAL (NULL, wrong row count), CC_E_RANGE (unknown table, tables
 * above CC_MAX_TOTAL_ROWS / CC_MAX_TOTAL_CELLS), CC_E_NOMEM, CC_E_HIP.
 */
cc_status cc_load(cc_ctx *ctx, uint32_t table_id, const int64_t *rows, uint64_t n_rows, int rows_on_device);

/*
 * Copy a table's current contents out (row-major) into out: n_rows x
 * n_fields int64 values, host memory, or device memory when out_on_device is
 * non-zero.  The final-state snapshot that verification compares (paper
 * Section 3.4, "Measurements and Verification").  Errors: CC_E_INVAL,
 * CC_E_RANGE (unknown table), CC_E_STATE (not loaded), CC_E_HIP.
 */
cc_status cc_read_table(cc_ctx *ctx, uint32_t table_id, int64_t *out, int out_on_device);

/*
 * Validate a batch of n_txns transactions over n_ops operations and stage it
 * in device memory for `scheme`: a batch whose read and write sets are fixed
 * before execution, over existing rows only (paper Section 4.1,
 * "Constraints"; the batch model of Section 3.3).  txns / ops are host
 * arrays (on_device = 0: validated on the host, packed and copied), or
 * device pointers on the context's device (on_device != 0, e.g. torch
 * tensors' data_ptr(): an ingest kernel validates them with the same rules
 * and the same status codes and packs them into the engine's layout, on the
 * context's stream).  Either way the arrays are read during the call only;
 * the caller keeps ownership and may reuse them once it returns.  Errors:
 * CC_E_INVAL (bad scheme/kind, op ranges outside the ops array, two
 * transactions sharing an op, WRITE_SLOT source not earlier, too many ops in
 * a txn, reserved not 0; for CC_GACCO and CC_GPUTX, a transaction whose
 * first_op is below the previous one's), CC_E_RANGE, CC_E_DUPROW,
 * CC_E_NOMEM.  When several transactions are malformed, the status is that
 * of the lowest-numbered one.  *batch_id receives a handle valid until
 * cc_release_batch or cc_destroy.  Zero transactions is a valid (empty)
 * batch.
 */
cc_status cc_submit_batch(cc_ctx *ctx, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                          int scheme, int on_device, uint64_t *batch_id);

/*
 * Give a table a sorted-array index (paper Section 3.4 "Index": the indexed
 * column is sorted and copied to device memory with the row ids; a lookup is
 * a search of the sorted array).  keys[i] (host array, n == the table's row
 * count) is row i's key; keys must be distinct and below INT64_MAX (the
 * padding value).  The engine sorts the (key, row) pairs on the host, copies
 * them to the device and builds a static 16-way search tree over them (each
 * level holds the largest key of every 16-key node below it; used with
 * CC_RUN_INDEX_TREE).  Load-time work, not part of any run.  Errors:
 * CC_E_INVAL (duplicate or reserved key, wrong n), CC_E_RANGE, CC_E_STATE
 * (a keyed batch is still submitted: release it first).
 */
cc_status cc_create_index(cc_ctx *ctx, uint32_t table_id, const int64_t *keys, uint64_t n);

/*
 * cc_submit_batch for batches that name rows by key: for an op on a table
 * with an index, op_keys[i] is its key and ops[i].row must be 0; ops on other
 * tables use ops[i].row as usual (their op_keys entry is ignored).  Row-group
 * and duplicate checks compare keys.  Each cc_run first looks every key up on
 * the device (after CC initialisation, inside the measured window:
 * CC_STAT_INDEX_NS) and returns CC_E_RANGE, with nothing executed, if a key
 * names no row.  op_keys is a host array of n_ops entries, copied.
 */
cc_status cc_submit_batch_keyed(cc_ctx *ctx, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                                const int64_t *op_keys, int scheme, int on_device, uint64_t *batch_id);

/*
 * For a keyed batch after a run: rows[i] (host array, n_ops entries) is the
 * row within its table that op i accessed -- the lookup's result for keyed
 * ops, ops[i].row for the others.  CC_E_STATE for a batch without keyed ops
 * or not yet run.
 */
cc_status cc_fetch_rows(cc_ctx *ctx, uint64_t batch_id, uint32_t *rows);

/*
 * The OCC hot-row engine's plan for a batch, made at submission (see
 * CC_RUN_HOT_ENGINE): rows (host array of CC_ENGINE_MAX_ROWS entries)
 * receives the engine rows as global row ids -- the table's first row in the
 * shared row space plus the row, tables in creation order -- most written
 * first; *n_rows their count (0: no engine for this batch: not OCC, keyed,
 * static, or nothing written often enough); *n_txns the transactions that
 * write one of them; *by_default 1 if no row left out of the engine is
 * written more than a quarter as often as the most written one -- one of the
 * conditions under which cc_run uses the engine without CC_RUN_HOT_ENGINE
 * (see there).  Host-side; no device work.
 */
#define CC_ENGINE_MAX_ROWS 32
cc_status cc_engine_plan(cc_ctx *ctx, uint64_t batch_id, uint32_t *rows, uint32_t *n_rows, uint64_t *n_txns,
                         int *by_default);

/*
 * Host-only validation of a batch against table shapes (n_tables tables of
 * n_rows[t] x n_fields[t]), with exactly the checks cc_submit_batch applies.
 * Touches no device; usable without a GPU.  Returns CC_OK or the status
 * cc_submit_batch would return for the same arrays.
 */
cc_status cc_check_batch(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields, const cc_txn *txns,
                         uint64_t n_txns, const cc_op *ops, uint64_t n_ops, int scheme);

/*
 * Execute a submitted batch and block until it finishes.  The run resets the
 * scheme's control words (CC initialisation, inside the measured window as in
 * the paper's throughput definition, Section 4.1 "Metric Selection") and then
 * runs every transaction until it commits.  A batch may be run repeatedly;
 * each run applies its writes to the current tables.
 * params may be NULL (all defaults).  Returns CC_E_LIVELOCK if a transaction
 * exhausted max_attempts (its status stays CC_PENDING and it left no writes),
 * CC_E_TS_OVERFLOW if a timestamp field overflowed.  CC_GACCO and CC_GPUTX
 * run every transaction exactly once after their preprocessing
 * (CC_STAT_PREP_NS; for GPUTx it includes the rank pass and the sort into
 * K-sets); they return CC_E_LIVELOCK only if a transaction waited more than
 * 4 s without progress, which a consistent lock table rules out.
 */
cc_status cc_run(cc_ctx *ctx, uint64_t batch_id, const cc_run_params *params);

/*
 * Host-only check of run parameters for a scheme: returns CC_OK, or the
 * status cc_run would return for these parameters before touching the
 * device (unknown mode or flag, lanes_per_txn not 1/4/16/64, waves_per_wg
 * above 16, a flag the scheme does not implement, CC_RUN_PRECHECK with
 * CC_RUN_NO_PRECHECK, wait_limit_us for a scheme without waits, a mode
 * GaccO / GPUTx do not run).  params may be NULL (defaults).  Usable without
 * a GPU.
 */
cc_status cc_check_run_params(int scheme, const cc_run_params *params);

/*
 * Copy the last run's per-transaction outcomes (n_txns entries) and per-op
 * read values (n_ops entries, indexed like the submitted ops array) out:
 * what the paper's verification consumes (Section 3.4, "Measurements and
 * Verification"), with the serial key in place of its event log.  Either
 * pointer may be NULL.  dst_on_device selects device destinations.  Errors:
 * CC_E_NOBATCH, CC_E_STATE (batch not run), CC_E_HIP.
 */
cc_status cc_fetch_outcomes(cc_ctx *ctx, uint64_t batch_id, cc_outcome *per_txn, int64_t *per_op_read,
                            int dst_on_device);

/*
 * Set the arrival time of every transaction of a batch, for CC_MODE_SERVE:
 * arrival_ns[t] is nanoseconds after the start of the run (CC
 * initialisation), non-decreasing in t, n == the batch's transaction count.
 * Host array; copied.  CC_E_INVAL on a decreasing or negative time.
 */
cc_status cc_set_arrivals(cc_ctx *ctx, uint64_t batch_id, const int64_t *arrival_ns, uint64_t n);

/*
 * Copy up to n counters (enum cc_stat order) of the batch's last run: the
 * paper's metrics (Section 4.1, "Metric Selection": throughput over the
 * window from CC initialisation to the last commit, abort rate) and its
 * breakdown of time into useful work, aborts and waiting (Section 3.4,
 * "Measurements and Verification").  Host memory.  Errors: CC_E_INVAL,
 * CC_E_NOBATCH.
 */
cc_status cc_stats(cc_ctx *ctx, uint64_t batch_id, uint64_t *counters, uint32_t n);

/* Free a batch's device buffers. */
cc_status cc_release_batch(cc_ctx *ctx, uint64_t batch_id);

/*
 * Allocation-free run, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  One call validates, packs and runs a batch that is already in
 * device memory and writes its outcomes into the caller's device arrays, as
 * cc_submit_batch (on_device = 1) + cc_run + cc_fetch_outcomes
 * (dst_on_device = 1) + cc_release_batch would, and allocates nothing.
 *
 *   txns, ops            device memory of the context's device, n_txns and
 *                        n_ops entries, as for cc_submit_batch; borrowed for
 *                        the call and not modified.
 *   per_txn, per_op_read device memory, n_txns and n_ops entries; the run's
 *                        outcomes and read values (entries of ops that no
 *                        transaction names are 0).
 *   scheme               CC_OCC, CC_2PL_NW, CC_2PL_WD, CC_TO or CC_TICTOC;
 *                        the others need buffers sized by the batch
 *                        (CC_E_INVAL).
 *   params               as for cc_run (NULL: defaults); CC_MODE_PLAIN only
 *                        and no CC_RUN_LATCH (CC_E_INVAL).
 *   counters             optional host array of n_counters entries that
 *                        receives the run's statistics (enum cc_stat order;
 *                        the latency percentiles are not computed: 0).
 * Limits: n_txns <= CC_STATIC_MAX_TXNS and n_ops <= CC_STATIC_MAX_OPS, else
 * CC_E_RANGE before anything touches the device.  The descriptors, the
 * pending list and the ingest words live in one 23 MiB array per device
 * (static device memory, held until the process ends).  Every call on a
 * device, from any context or thread, shares that array: calls that overlap
 * on one GPU race, and the caller must serialise them.  Each call clears what
 * it reads before using it.  Errors: as cc_submit_batch and cc_run; a
 * malformed batch is reported before any transaction runs.
 */
cc_status cc_run_static(cc_ctx *ctx, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                        int scheme, const cc_run_params *params, cc_outcome *per_txn, int64_t *per_op_read,
                        uint64_t *counters, uint32_t n_counters);

/*
 * Memory micro-benchmarks that measure the roofline of the transaction
 * kernels, whose work is random 8-byte accesses and 64-bit atomics (not
 * streaming, not arithmetic).  kind:
 *   CC_PROBE_STREAM        16-byte streaming copy over footprint_bytes (reads + writes)
 *   CC_PROBE_GATHER        n_ops random 8-byte agent-scope (coherent) loads
 *   CC_PROBE_GATHER_PLAIN  n_ops random 8-byte plain loads
 *   CC_PROBE_SCATTER       n_ops random 8-byte agent-scope stores
 *   CC_PROBE_ATOMIC        n_ops random 64-bit fetch_or (agent scope)
 *   CC_PROBE_SAME_WORD     n_ops 64-bit fetch_add on one word, every lane
 *   CC_PROBE_WAVE_COUNTER  n_ops / 64 fetch_adds on one word, one per wavefront
 *   CC_PROBE_HANDOFF       n_ops ping-pong rounds on one word between two
 *                          workgroups `peer` apart (peer 1: another XCD; 8: same XCD)
 *   CC_PROBE_COMMIT_HANDOFF n_ops rounds of the OCC commit critical section on
 *                          one row (lock, value read + ticket, validation read,
 *                          value store, publish), alternating between two
 *                          workgroups `peer` apart: ms / n_ops is the hot-row
 *                          hand-off time t_h
 *   CC_PROBE_ENGINE_HANDOFF n_ops rounds of the OCC hot-row engine's commit
 *                          critical section on one engine row (LDS lock, LDS
 *                          ticket, LDS validation load, LDS store and release),
 *                          alternating between two wavefronts of one workgroup:
 *                          ms / n_ops is the engine's t_h (peer is ignored)
 * Random addresses are uniform over the footprint_bytes / 8 words of the
 * probe's buffer (rounded down to a multiple of 4).  For the hand-off probes,
 * peer places the second side: 0 in the same workgroup (same CU), 8 in
 * another workgroup of the same XCD, 1 on another XCD (workgroups are dealt
 * round-robin to the 8 XCDs).  *ms receives the kernel time (HIP events).
 * Allocates and frees its own buffers.  CC_E_LIVELOCK if a hand-off turn
 * exceeded its bounded wait.
 */
enum cc_probe_kind {
  CC_PROBE_STREAM = 0,
  CC_PROBE_GATHER = 1,
  CC_PROBE_GATHER_PLAIN = 2,
  CC_PROBE_SCATTER = 3,
  CC_PROBE_ATOMIC = 4,
  CC_PROBE_SAME_WORD = 5,
  CC_PROBE_WAVE_COUNTER = 6,
  CC_PROBE_HANDOFF = 7,
  CC_PROBE_COMMIT_HANDOFF = 8,
  CC_PROBE_ENGINE_HANDOFF = 9
};
cc_status cc_probe(cc_ctx *ctx, int kind, uint64_t footprint_bytes, uint64_t n_ops, int peer, double *ms);

/*
 * The gather, plain-gather, scatter or atomic probe at the caller's word
 * indices: op i touches word indices[i] of a footprint_bytes buffer, so a
 * skewed distribution (the workload's Zipf rows) can be measured.  indices is
 * a host array of n entries, each below footprint_bytes / 8 rounded down to a
 * multiple of 4 (else CC_E_RANGE); it is copied to the device before the
 * timed kernel, which also streams it.  *ms receives the kernel time.
 */
cc_status cc_probe_indices(cc_ctx *ctx, int kind, uint64_t footprint_bytes, const uint64_t *indices, uint64_t n,
                           double *ms);

/* Device properties the engine uses: compute units, wall-clock rate (kHz). */
cc_status cc_device_info(cc_ctx *ctx, uint32_t *n_cu, uint32_t *wallclock_khz);

#ifdef __cplusplus
}
#endif

#endif /* CC_H_ */
