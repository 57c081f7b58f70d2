// C-ABI of the batch transaction engine: context, tables, batches, runs.
// Declarations and the contract of every call are in include/cc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "engine.h"

using namespace cce;

namespace {

struct Table {
  uint64_t n_rows;
  uint32_t n_fields;
  uint64_t row_base;   // first global row id
  uint64_t elem_base;  // first cell in the value arena
};

struct Batch {
  int scheme = 0;
  uint64_t n_txns = 0, n_ops = 0;
  uint32_t max_ops = 0;
  bool has_slot = false;
  DevOp *d_ops = nullptr;
  DevTxn *d_txns = nullptr;
  DevOutcome *d_out = nullptr;
  int64_t *d_reads = nullptr;
  uint32_t *d_list = nullptr;  // pending transactions between passes
  uint64_t *d_nodes = nullptr; // MVCC version arena: a 32-byte header (the ring counter), then node_slots x 4 words
  uint64_t node_slots = 0;
  bool keyed = false;            // some ops name their row by key (cc_submit_batch_keyed)
  int64_t *d_opkeys = nullptr;   // keyed batches: per-op key
  uint32_t *d_meta = nullptr;    // keyed batches: per-op keyed flag, table, field
  uint32_t *d_rows = nullptr;    // keyed batches: per-op row found by the last run's lookups
  uint32_t *d_rank = nullptr;    // GaccO: per row-group leader, its position in the sorted access table
  uint32_t *d_gscratch = nullptr;// GaccO, GPUTx: access-table and sort buffers
  uint32_t *d_tscratch = nullptr;// GPUTx: per-transaction ranks, sort buffers, K-set starts
  int64_t *d_arrival = nullptr;           // serving: arrival ticks per transaction
  std::vector<int64_t> arrival_ns;        // host copy, for latency statistics
  hipGraphExec_t epoch_graph = nullptr;  // captured epochs for the last epoch-mode parameters
  uint64_t epoch_key[4] = {0, 0, 0, 0};
  int epoch_grid = 0;
  bool ran = false;
  uint64_t stats[CC_N_STATS] = {};
  // counted at submission (find_hot_rows): writes to the most written row,
  // and the most written rows (most first); hot_known is false for a batch
  // nobody counted (cc_run_static), which then runs with the contended defaults
  bool hot_known = false;
  uint64_t hot_writes = 0;
  uint32_t n_hot = 0;
  uint32_t hot_rows[HOT_MAX] = {};
  // OCC hot-row engine, planned at submission (plan_engine): its rows, and
  // d_part = the transactions that write one of them (n_eng_txns), then the
  // others; eng_gain: every row left out is written at most a quarter as often
  // as the most written row
  EngineArgs eng{};
  uint64_t n_eng_txns = 0;
  bool eng_gain = false;
  uint32_t *d_part = nullptr;
  EngineDesc *d_eng_desc = nullptr;  // the engine's transactions with their first op and op count
  std::vector<uint32_t> eng_part;  // host copies until the upload
  std::vector<EngineDesc> eng_desc;
};

}  // namespace

struct DevIndex {
  int64_t *keys = nullptr;
  uint32_t *rows = nullptr;
  int64_t *tree = nullptr;
  IndexDesc desc{};
};

struct cc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_cu = 0;
  uint32_t wallclock_khz = 0;
  std::vector<Table> tables;
  bool frozen = false;
  uint64_t total_rows = 0, total_cells = 0;
  int64_t *d_data = nullptr;
  uint64_t *d_words = nullptr;
  uint64_t *d_aux = nullptr;
  Ctl *d_ctl = nullptr;
  std::vector<DevIndex> indexes;      // per table (empty entries: no index)
  IndexDesc *d_idx = nullptr;         // device copy of every table's IndexDesc
  uint32_t *d_latch = nullptr;        // CC_RUN_LATCH: one latch per global row
  uint64_t *d_kstate = nullptr;       // GPUTx: per-row rank state
  uint64_t *d_ingest = nullptr;       // device-side batch ingest: reduced results
  unsigned char *d_static = nullptr;  // cc_run_static: this device's static scratch (never freed)
  std::map<uint64_t, Batch> batches;
  uint64_t next_batch = 1;
  hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  std::string err;
};

namespace {

thread_local std::string g_init_err;

cc_status fail(cc_ctx *c, cc_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

cc_status hip_fail(cc_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(c, CC_E_NOMEM, m);
  return fail(c, CC_E_HIP, m);
}

#define HIP_OR(ctx, call)                              \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

bool activate(cc_ctx *c) { return hipSetDevice(c->device) == hipSuccess; }

cc_status freeze(cc_ctx *c) {
  if (c->frozen) return CC_OK;
  if (c->tables.empty()) return fail(c, CC_E_STATE, "no tables declared");
  uint64_t rows = 0, cells = 0;
  for (auto &t : c->tables) {
    t.row_base = rows;
    t.elem_base = cells;
    rows += t.n_rows;
    cells += t.n_rows * t.n_fields;
  }
  if (rows > CC_MAX_TOTAL_ROWS || cells > CC_MAX_TOTAL_CELLS) return fail(c, CC_E_RANGE, "tables too large");
  c->total_rows = rows;
  c->total_cells = cells;
  // all or nothing: a failed step frees what it allocated, so a later call can try again
  int64_t *data = nullptr;
  uint64_t *words = nullptr;
  hipError_t e = hipMalloc(&data, std::max<uint64_t>(cells, 1) * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&words, std::max<uint64_t>(rows, 1) * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemsetAsync(data, 0, std::max<uint64_t>(cells, 1) * sizeof(int64_t), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    if (data) (void)hipFree(data);
    if (words) (void)hipFree(words);
    return hip_fail(c, e, "table allocation");
  }
  c->d_data = data;
  c->d_words = words;
  c->frozen = true;
  return CC_OK;
}

cc_status launch_error(cc_ctx *c, hipError_t e) {
  if (e == hipErrorInvalidValue) return fail(c, CC_E_INVAL, "scheme or (lanes_per_txn, ops per txn) not supported");
  if (e == hipErrorInvalidConfiguration)
    return fail(c, CC_E_INVAL, "waves_per_wg too large for the register slots this lanes_per_txn needs");
  return hip_fail(c, e, "transaction kernel launch");
}

// Resolve a keyed batch's keys on the device, after CC initialisation and
// inside the run's window; *ms receives the lookup kernel's time.
cc_status resolve_keys(cc_ctx *c, Batch &b, const cc_run_params &p, float *ms) {
  HIP_OR(c, hipEventRecord(c->ev[6], c->stream));
  HIP_OR(c, launch_index_lookup(c->stream, (p.flags & CC_RUN_INDEX_TREE) != 0, b.d_opkeys, b.d_meta, b.d_ops,
                                b.d_rows, b.n_ops, c->d_idx, c->d_ctl));
  HIP_OR(c, hipEventRecord(c->ev[7], c->stream));
  uint64_t miss = 0;
  HIP_OR(c, hipMemcpyAsync(&miss, &c->d_ctl->stats[DS_INDEX_MISS], sizeof miss, hipMemcpyDeviceToHost, c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  HIP_OR(c, hipEventElapsedTime(ms, c->ev[6], c->ev[7]));
  if (miss) return fail(c, CC_E_RANGE, std::to_string(miss) + " keys name no row of their table's index");
  return CC_OK;
}

void free_batch(Batch &b) {
  if (b.d_ops) (void)hipFree(b.d_ops);
  if (b.d_txns) (void)hipFree(b.d_txns);
  if (b.d_out) (void)hipFree(b.d_out);
  if (b.d_reads) (void)hipFree(b.d_reads);
  if (b.d_list) (void)hipFree(b.d_list);
  if (b.d_part) (void)hipFree(b.d_part);
  b.d_part = nullptr;
  if (b.d_eng_desc) (void)hipFree(b.d_eng_desc);
  b.d_eng_desc = nullptr;
  if (b.d_nodes) (void)hipFree(b.d_nodes);
  if (b.d_opkeys) (void)hipFree(b.d_opkeys);
  if (b.d_meta) (void)hipFree(b.d_meta);
  if (b.d_rows) (void)hipFree(b.d_rows);
  b.d_opkeys = nullptr;
  b.d_meta = nullptr;
  b.d_rows = nullptr;
  if (b.d_rank) (void)hipFree(b.d_rank);
  if (b.d_gscratch) (void)hipFree(b.d_gscratch);
  if (b.d_tscratch) (void)hipFree(b.d_tscratch);
  b.d_tscratch = nullptr;
  b.d_rank = nullptr;
  b.d_gscratch = nullptr;
  if (b.epoch_graph) (void)hipGraphExecDestroy(b.epoch_graph);
  if (b.d_arrival) (void)hipFree(b.d_arrival);
  b.d_arrival = nullptr;
  b.epoch_graph = nullptr;
  b.d_list = nullptr;
  b.d_nodes = nullptr;
  b.node_slots = 0;
  b.d_ops = nullptr;
  b.d_txns = nullptr;
  b.d_out = nullptr;
  b.d_reads = nullptr;
}

// Percentile of committed commit times (host side, after a run).
void latency_percentiles(std::vector<cc_outcome> &o, uint64_t *p50, uint64_t *p99) {
  std::vector<int64_t> lat;
  lat.reserve(o.size());
  for (auto &x : o)
    if (x.status == CC_COMMITTED) lat.push_back(x.commit_ns);
  if (lat.empty()) {
    *p50 = *p99 = 0;
    return;
  }
  auto pick = [&](double q) {
    size_t i = (size_t)(q * (double)(lat.size() - 1) + 0.5);
    std::nth_element(lat.begin(), lat.begin() + i, lat.end());
    return (uint64_t)lat[i];
  };
  *p50 = pick(0.50);
  *p99 = pick(0.99);
}

}  // namespace

extern "C" {

const char *cc_version(void) { return "cc-gfx950 0.1"; }

const char *cc_strerror(cc_status s) {
  switch (s) {
    case CC_OK: return "ok";
    case CC_E_INVAL: return "invalid argument";
    case CC_E_RANGE: return "out of range";
    case CC_E_DUPROW: return "duplicate row access within a transaction";
    case CC_E_NOMEM: return "out of memory";
    case CC_E_TS_OVERFLOW: return "timestamp overflow";
    case CC_E_LIVELOCK: return "transactions still pending (attempt or epoch limit reached)";
    case CC_E_HIP: return "HIP runtime error";
    case CC_E_NODEV: return "no usable gfx950 device";
    case CC_E_STATE: return "call out of order";
    case CC_E_NOBATCH: return "unknown batch";
    default: return "unknown status";
  }
}

const char *cc_last_error(const cc_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_err.c_str(); }

cc_status cc_init(cc_ctx **out, const cc_config *cfg) {
  if (!out) return CC_E_INVAL;
  *out = nullptr;
  g_init_err.clear();
  int dev = cfg ? cfg->device : 0;
  if (cfg && cfg->flags != 0) {
    g_init_err = "cc_config.flags must be 0";
    return CC_E_INVAL;
  }
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    g_init_err = "no HIP device";
    return CC_E_NODEV;
  }
  if (dev < 0 || dev >= n) {
    g_init_err = "device ordinal out of range";
    return CC_E_NODEV;
  }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    g_init_err = "hipGetDeviceProperties failed";
    return CC_E_NODEV;
  }
  if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
    g_init_err = std::string("device is ") + p.gcnArchName + ", the engine is built for gfx950";
    return CC_E_NODEV;
  }
  cc_ctx *c = new (std::nothrow) cc_ctx();
  if (!c) return CC_E_NOMEM;
  c->device = dev;
  c->stream = cfg ? (hipStream_t)cfg->stream : nullptr;
  c->n_cu = p.multiProcessorCount;
  if (!c->stream) {
    // a stream of our own (default priority), so that runs can be captured
    if (hipSetDevice(dev) != hipSuccess || hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      g_init_err = "hipStreamCreate failed";
      return CC_E_HIP;
    }
    c->own_stream = true;
  }
  int khz = 0;
  if (hipSetDevice(dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
    delete c;
    g_init_err = "cannot read the device wall-clock rate";
    return CC_E_HIP;
  }
  c->wallclock_khz = (uint32_t)khz;
  if (hipMalloc(&c->d_ctl, sizeof(Ctl)) != hipSuccess) {
    delete c;
    g_init_err = "hipMalloc of the control block failed";
    return CC_E_NOMEM;
  }
  for (auto &e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      cc_destroy(c);
      g_init_err = "hipEventCreate failed";
      return CC_E_HIP;
    }
  }
  // the allocation-free run's scratch on this device (the device is current)
  void *sp = nullptr;
  const hipError_t se = static_scratch_address(dev, &sp);
  if (se != hipSuccess) {
    cc_destroy(c);
    g_init_err = std::string("device address of the static scratch: ") + hipGetErrorString(se);
    return CC_E_HIP;
  }
  c->d_static = (unsigned char *)sp;
  *out = c;
  return CC_OK;
}

cc_status cc_destroy(cc_ctx *c) {
  if (!c) return CC_OK;
  activate(c);
  (void)hipStreamSynchronize(c->stream);
  for (auto &kv : c->batches) free_batch(kv.second);
  for (auto &ix : c->indexes) {
    if (ix.keys) (void)hipFree(ix.keys);
    if (ix.rows) (void)hipFree(ix.rows);
    if (ix.tree) (void)hipFree(ix.tree);
  }
  if (c->d_idx) (void)hipFree(c->d_idx);
  if (c->d_latch) (void)hipFree(c->d_latch);
  if (c->d_kstate) (void)hipFree(c->d_kstate);
  if (c->d_ingest) (void)hipFree(c->d_ingest);
  if (c->d_data) (void)hipFree(c->d_data);
  if (c->d_words) (void)hipFree(c->d_words);
  if (c->d_aux) (void)hipFree(c->d_aux);
  if (c->d_ctl) (void)hipFree(c->d_ctl);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return CC_OK;
}

cc_status cc_probe(cc_ctx *c, int kind, uint64_t footprint_bytes, uint64_t n_ops, int peer, double *ms) {
  if (!c || !ms) return CC_E_INVAL;
  if (kind < CC_PROBE_STREAM || kind > CC_PROBE_ENGINE_HANDOFF) return fail(c, CC_E_INVAL, "unknown probe");
  const bool pair = kind == CC_PROBE_HANDOFF || kind == CC_PROBE_COMMIT_HANDOFF;
  if (footprint_bytes < 4096 || (pair && (peer < 0 || peer > 64)))
    return fail(c, CC_E_INVAL, "bad probe size or peer");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  uint64_t err = 0;
  hipError_t e = run_probe(c->stream, kind, footprint_bytes, n_ops, peer, nullptr, ms, &err, c->n_cu);
  if (e != hipSuccess) return hip_fail(c, e, "probe");
  if (err) return fail(c, CC_E_LIVELOCK, "hand-off turn exceeded its bounded wait");
  return CC_OK;
}

cc_status cc_probe_indices(cc_ctx *c, int kind, uint64_t footprint_bytes, const uint64_t *indices, uint64_t n,
                           double *ms) {
  if (!c || !ms || (n && !indices)) return CC_E_INVAL;
  if (kind != CC_PROBE_GATHER && kind != CC_PROBE_GATHER_PLAIN && kind != CC_PROBE_SCATTER && kind != CC_PROBE_ATOMIC)
    return fail(c, CC_E_INVAL, "cc_probe_indices runs the gather, scatter and atomic probes");
  if (footprint_bytes < 4096) return fail(c, CC_E_INVAL, "bad probe size");
  const uint64_t words = footprint_bytes / sizeof(uint64_t) / 4 * 4;
  for (uint64_t i = 0; i < n; ++i)
    if (indices[i] >= words) return fail(c, CC_E_RANGE, "index beyond the probe's footprint");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  uint64_t err = 0;
  hipError_t e = run_probe(c->stream, kind, footprint_bytes, n, 1, indices, ms, &err, c->n_cu);
  if (e != hipSuccess) return hip_fail(c, e, "probe");
  return CC_OK;
}

cc_status cc_device_info(cc_ctx *c, uint32_t *n_cu, uint32_t *khz) {
  if (!c) return CC_E_INVAL;
  if (n_cu) *n_cu = (uint32_t)c->n_cu;
  if (khz) *khz = c->wallclock_khz;
  return CC_OK;
}

cc_status cc_create_table(cc_ctx *c, uint64_t n_rows, uint32_t n_fields, uint32_t *table_id) {
  if (!c || !table_id) return CC_E_INVAL;
  if (c->frozen) return fail(c, CC_E_STATE, "tables must be declared before the first cc_load");
  if (n_rows == 0 || n_fields == 0 || n_fields > 256) return fail(c, CC_E_INVAL, "bad table shape");
  if (c->tables.size() >= CC_MAX_TABLES) return fail(c, CC_E_RANGE, "too many tables");
  c->tables.push_back(Table{n_rows, n_fields, 0, 0});
  *table_id = (uint32_t)(c->tables.size() - 1);
  return CC_OK;
}

cc_status cc_load(cc_ctx *c, uint32_t tid, const int64_t *rows, uint64_t n_rows, int on_device) {
  if (!c || !rows) return CC_E_INVAL;
  if (tid >= c->tables.size()) return fail(c, CC_E_RANGE, "unknown table");
  if (n_rows != c->tables[tid].n_rows) return fail(c, CC_E_INVAL, "row count differs from the table's");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  cc_status st = freeze(c);
  if (st) return st;
  const Table &t = c->tables[tid];
  HIP_OR(c, hipMemcpyAsync(c->d_data + t.elem_base, rows, t.n_rows * t.n_fields * sizeof(int64_t),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  return CC_OK;
}

cc_status cc_read_table(cc_ctx *c, uint32_t tid, int64_t *out, int on_device) {
  if (!c || !out) return CC_E_INVAL;
  if (tid >= c->tables.size()) return fail(c, CC_E_RANGE, "unknown table");
  if (!c->frozen) return fail(c, CC_E_STATE, "table not loaded");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  const Table &t = c->tables[tid];
  HIP_OR(c, hipMemcpyAsync(out, c->d_data + t.elem_base, t.n_rows * t.n_fields * sizeof(int64_t),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  return CC_OK;
}

}  // extern "C"

namespace {

// Validate a batch against table shapes and build its device descriptors.
cc_status validate_and_pack(cc_ctx *c, const std::vector<Table> &tables, const cc_txn *txns, uint64_t n_txns,
                            const cc_op *ops, uint64_t n_ops, std::vector<DevOp> *dops_out,
                            std::vector<DevTxn> *dtx_out, uint32_t *max_ops_out, bool *has_slot_out,
                            bool *txn_ordered_out, const int64_t *op_keys = nullptr,
                            const std::vector<bool> *indexed = nullptr) {
  if ((n_txns && !txns) || (n_ops && !ops)) return fail(c, CC_E_INVAL, "null array");
  if (n_txns > 0xFFFFFFFFull || n_ops > 0xFFFFFFFFull) return fail(c, CC_E_RANGE, "batch too large");
  std::vector<DevOp> dummy_ops;
  std::vector<DevTxn> dummy_tx;
  std::vector<DevOp> &dops = dops_out ? *dops_out : dummy_ops;
  std::vector<DevTxn> &dtx = dtx_out ? *dtx_out : dummy_tx;
  // operations no transaction refers to are marked as followers: they never
  // enter GaccO's access table
  dops.assign(n_ops, DevOp{FOLLOWER_BIT, 0, 0});
  bool txn_ordered = true;  // every transaction's ops come after the previous one's
  dtx.assign(n_txns, DevTxn{0, 0});
  std::vector<uint8_t> used(n_ops, 0);  // every op belongs to at most one transaction
  std::vector<std::pair<uint32_t, int64_t>> keys;  // (table, row or key) of row leaders, for the duplicate check
  uint32_t max_ops = 0;
  bool has_slot = false;
  for (uint64_t t = 0; t < n_txns; ++t) {
    const cc_txn &x = txns[t];
    if (x.reserved != 0) return fail(c, CC_E_INVAL, "cc_txn.reserved must be 0");
    if (x.n_ops > CC_MAX_OPS_PER_TXN) return fail(c, CC_E_INVAL, "transaction has too many ops");
    if (x.first_op > n_ops || x.n_ops > n_ops - x.first_op) return fail(c, CC_E_INVAL, "op range outside ops");
    if (t > 0 && x.first_op < txns[t - 1].first_op) txn_ordered = false;
    for (uint32_t i = 0; i < x.n_ops; ++i) {
      if (used[x.first_op + i]) return fail(c, CC_E_INVAL, "transactions share operations");
      used[x.first_op + i] = 1;
    }
    max_ops = std::max(max_ops, x.n_ops);
    keys.clear();
    uint32_t group_start = 0;
    bool group_written = false;
    // an op's row identity: its key on a table with an index (keyed batch), else its row
    auto keyed = [&](const cc_op &o) { return op_keys && indexed && o.table < indexed->size() && (*indexed)[o.table]; };
    auto ident = [&](uint32_t k) -> int64_t {
      const cc_op &o = ops[x.first_op + k];
      return keyed(o) ? op_keys[x.first_op + k] : (int64_t)o.row;
    };
    for (uint32_t i = 0; i < x.n_ops; ++i) {
      const cc_op &o = ops[x.first_op + i];
      if (o.table >= tables.size()) return fail(c, CC_E_RANGE, "op table out of range");
      const Table &tb = tables[o.table];
      const bool kd = keyed(o);
      if (kd && o.row != 0) return fail(c, CC_E_INVAL, "an op on an indexed table names its row by key; row must be 0");
      if ((!kd && o.row >= tb.n_rows) || o.field >= tb.n_fields) return fail(c, CC_E_RANGE, "op row/field out of range");
      if (o.kind > CC_WRITE_SLOT) return fail(c, CC_E_INVAL, "unknown op kind");
      if (o.kind == CC_WRITE_SLOT) {
        has_slot = true;
        if ((uint32_t)(o.arg & 0xFF) >= i) return fail(c, CC_E_INVAL, "WRITE_SLOT source is not an earlier op");
      }
      const bool follower = i > 0 && ops[x.first_op + i - 1].table == o.table && ident(i - 1) == ident(i);
      if (!follower) {
        for (uint32_t j = group_start; j < i; ++j)
          if (group_written) dops[x.first_op + j].rowk |= WRITTEN_BIT;
        group_start = i;
        group_written = false;
        keys.emplace_back((uint32_t)o.table, ident(i));
      } else {
        for (uint32_t j = group_start; j < i; ++j)
          if (ops[x.first_op + j].field == o.field) return fail(c, CC_E_DUPROW, "field repeated within a txn");
      }
      group_written |= o.kind != CC_READ;
      // keyed ops get their row and cell from the lookup at the start of each run
      const uint64_t grow = kd ? 0 : tb.row_base + o.row;
      DevOp d;
      d.rowk = (uint32_t)grow | ((uint32_t)o.kind << KIND_SHIFT) | (follower ? FOLLOWER_BIT : 0u);
      d.elem = kd ? 0u : (uint32_t)(tb.elem_base + (uint64_t)o.row * tb.n_fields + o.field);
      d.arg = o.arg;
      dops[x.first_op + i] = d;
    }
    for (uint32_t j = group_start; j < x.n_ops; ++j)
      if (group_written) dops[x.first_op + j].rowk |= WRITTEN_BIT;
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
      return fail(c, CC_E_DUPROW, "row accessed twice (non-adjacent) within a txn");
    dtx[t].first = (uint32_t)x.first_op;
    dtx[t].n = x.n_ops;
  }
  if (max_ops_out) *max_ops_out = max_ops;
  if (has_slot_out) *has_slot_out = has_slot;
  if (txn_ordered_out) *txn_ordered_out = txn_ordered;
  return CC_OK;
}

std::vector<Table> layout_tables(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields) {
  std::vector<Table> v;
  uint64_t rows = 0, cells = 0;
  for (uint32_t t = 0; t < n_tables; ++t) {
    v.push_back(Table{n_rows[t], n_fields[t], rows, cells});
    rows += n_rows[t];
    cells += n_rows[t] * n_fields[t];
  }
  return v;
}

// GaccO run: CC initialisation, preprocessing (access table, sort, lock
// table), one execution pass.  Every transaction runs exactly once.
constexpr uint64_t GACCO_WAIT_LIMIT_MS = 4000;

// Wall-clock ticks a waiting team may go without progress before it stops
// the run (cc_run_params.wait_limit_us; 0 = GACCO_WAIT_LIMIT_MS).
uint64_t wait_limit_ticks(const cc_ctx *c, const cc_run_params &p) {
  if (p.wait_limit_us == 0) return (uint64_t)c->wallclock_khz * GACCO_WAIT_LIMIT_MS;
  return std::max<uint64_t>(1, p.wait_limit_us * c->wallclock_khz / 1000ull);
}

// (mode and flags were checked by check_run_params)
cc_status run_gacco(cc_ctx *c, Batch &b, const cc_run_params &p, uint32_t lanes, uint32_t wpw) {
  GaccoArgs a{};
  a.ops = b.d_ops;
  a.txns = b.d_txns;
  a.n_txns = b.n_txns;
  a.rank = b.d_rank;
  a.data = c->d_data;
  a.words = c->d_words;
  a.out = b.d_out;
  a.reads = b.d_reads;
  a.ctl = c->d_ctl;
  a.wait_limit_ticks = wait_limit_ticks(c, p);
  const uint64_t poll_ns = p.backoff_ns ? p.backoff_ns : 200;
  a.poll_ticks = (uint32_t)std::max<uint64_t>(1, poll_ns * c->wallclock_khz / 1000000ull);
  a.ns_per_tick_q16 = (uint32_t)((1000000ull << 16) / c->wallclock_khz);
  a.has_slot = b.has_slot ? 1u : 0u;
  a.shared = (p.flags & CC_RUN_SHARED_READS) ? 1u : 0u;
  const bool strict = (p.flags & CC_RUN_STRICT_FENCES) != 0;

  HIP_OR(c, hipEventRecord(c->ev[0], c->stream));
  // the lock table sets the word of every accessed row, so words need no clearing
  HIP_OR(c, launch_init(c->stream, c->d_words, 0, nullptr, 0, b.d_out, b.n_txns, c->d_ctl, p.ts_start));
  float ms_index = 0;
  if (b.keyed) {
    cc_status st = resolve_keys(c, b, p, &ms_index);
    if (st) return st;
  }
  HIP_OR(c, hipEventRecord(c->ev[4], c->stream));
  HIP_OR(c, gacco_prepare(c->stream, b.d_ops, b.n_ops, (uint32_t)c->total_rows, c->d_words, b.d_rank, b.d_gscratch,
                          c->d_ctl, a.shared ? PREP_SHARED : PREP_TURNS));
  HIP_OR(c, hipEventRecord(c->ev[5], c->stream));
  HIP_OR(c, hipEventRecord(c->ev[1], c->stream));
  int grid_used = 0;
  if (b.n_txns) {
    hipError_t e = launch_gacco(c->stream, (int)lanes, (int)b.max_ops, (int)wpw, (int)p.grid, strict, a, c->n_cu,
                                &grid_used);
    if (e != hipSuccess) return launch_error(c, e);
  }
  HIP_OR(c, hipEventRecord(c->ev[2], c->stream));
  HIP_OR(c, hipEventRecord(c->ev[3], c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  Ctl h{};
  HIP_OR(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  float ms_run = 0, ms_prep = 0, ms_kernel = 0;
  HIP_OR(c, hipEventElapsedTime(&ms_run, c->ev[0], c->ev[3]));
  HIP_OR(c, hipEventElapsedTime(&ms_prep, c->ev[4], c->ev[5]));
  HIP_OR(c, hipEventElapsedTime(&ms_kernel, c->ev[1], c->ev[2]));
  std::memset(b.stats, 0, sizeof(b.stats));
  b.stats[CC_STAT_COMMITTED] = h.stats[DS_COMMITTED];
  b.stats[CC_STAT_ATTEMPTS] = h.stats[DS_ATTEMPTS];
  b.stats[CC_STAT_KERNEL_NS] = (uint64_t)((double)ms_kernel * 1e6);
  b.stats[CC_STAT_RUN_NS] = (uint64_t)((double)ms_run * 1e6);
  b.stats[CC_STAT_PREP_NS] = (uint64_t)((double)ms_prep * 1e6);
  b.stats[CC_STAT_INDEX_NS] = (uint64_t)((double)ms_index * 1e6);
  b.stats[CC_STAT_MAX_ATTEMPTS] = h.stats[DS_MAX_ATTEMPTS];
  b.stats[CC_STAT_PASSES] = b.n_txns ? 1 : 0;
  b.stats[CC_STAT_GRID] = (uint64_t)grid_used;
  const double ns_per_tick = 1e6 / (double)c->wallclock_khz;
  b.stats[CC_STAT_T_USEFUL_NS] = (uint64_t)((double)h.stats[DS_T_USEFUL] * ns_per_tick);
  b.stats[CC_STAT_T_WAIT_NS] = (uint64_t)((double)h.stats[DS_T_WAIT] * ns_per_tick);
  b.ran = true;
  if (b.n_txns) {
    std::vector<cc_outcome> o(b.n_txns);
    HIP_OR(c, hipMemcpy(o.data(), b.d_out, b.n_txns * sizeof(cc_outcome), hipMemcpyDeviceToHost));
    latency_percentiles(o, &b.stats[CC_STAT_LAT_P50_NS], &b.stats[CC_STAT_LAT_P99_NS]);
  }
  if (h.stop) return fail(c, CC_E_LIVELOCK, "CC_GACCO: a transaction waited past the limit for its turn on a row");
  if (h.stats[DS_COMMITTED] != b.n_txns) return fail(c, CC_E_LIVELOCK, "CC_GACCO: not every transaction ran");
  return CC_OK;
}

uint64_t gputx_scratch_words(uint64_t n_txns) { return 3 * n_txns + 1 + radix_sort_scratch_words(n_txns); }

// GPUTx run: CC initialisation, [index lookups], preprocessing shared with
// GaccO, the rank pass, the sort into K-sets, and the K-set-ordered
// execution.  Every transaction runs exactly once.
// (mode and flags were checked by check_run_params)
cc_status run_gputx(cc_ctx *c, Batch &b, const cc_run_params &p, uint32_t lanes, uint32_t wpw) {
  if (!c->d_kstate) HIP_OR(c, hipMalloc(&c->d_kstate, std::max<uint64_t>(c->total_rows, 1) * sizeof(uint64_t)));
  const uint64_t n = b.n_txns;
  uint32_t *txn_rank = b.d_tscratch, *iota = txn_rank + n, *kstart = iota + n, *sort_scratch = kstart + n + 1;
  GputxArgs a{};
  a.ops = b.d_ops;
  a.txns = b.d_txns;
  a.n_txns = n;
  a.rank = b.d_rank;
  a.words = c->d_words;
  a.kstate = c->d_kstate;
  a.txn_rank = txn_rank;
  a.kstart = kstart;
  a.data = c->d_data;
  a.out = b.d_out;
  a.reads = b.d_reads;
  a.ctl = c->d_ctl;
  a.wait_limit_ticks = wait_limit_ticks(c, p);
  const uint64_t poll_ns = p.backoff_ns ? p.backoff_ns : 200;
  a.poll_ticks = (uint32_t)std::max<uint64_t>(1, poll_ns * c->wallclock_khz / 1000000ull);
  a.ns_per_tick_q16 = (uint32_t)((1000000ull << 16) / c->wallclock_khz);
  a.has_slot = b.has_slot ? 1u : 0u;
  // the rank pass keeps each row's rank state in its turn word when both fit
  // (rank + 1 in 20 bits, a row's place in its list in 24)
  const bool packed = n < (1ull << 20) && b.n_ops < (1ull << 24);
  a.packed = packed ? 1u : 0u;
  const bool strict = (p.flags & CC_RUN_STRICT_FENCES) != 0;

  HIP_OR(c, hipEventRecord(c->ev[0], c->stream));
  HIP_OR(c, launch_init(c->stream, c->d_words, 0, nullptr, 0, b.d_out, n, c->d_ctl, 0));
  float ms_index = 0;
  if (b.keyed) {
    cc_status st = resolve_keys(c, b, p, &ms_index);
    if (st) return st;
  }
  HIP_OR(c, hipEventRecord(c->ev[4], c->stream));
  HIP_OR(c, gacco_prepare(c->stream, b.d_ops, b.n_ops, (uint32_t)c->total_rows, c->d_words, b.d_rank, b.d_gscratch,
                          c->d_ctl, packed ? PREP_LOCAL : PREP_TURNS));
  int grid_used = 0;
  if (n) {
    HIP_OR(c, gputx_init_state(c->stream, c->d_kstate, packed ? 0 : c->total_rows, iota, n));
    HIP_OR(c, gputx_reset(c->stream, c->d_ctl));
    hipError_t e = launch_gputx_pass(c->stream, false, (int)lanes, (int)b.max_ops, (int)wpw, (int)p.grid, strict, a,
                                     c->n_cu, &grid_used);
    if (e != hipSuccess) return launch_error(c, e);
    uint32_t *sk = nullptr, *sv = nullptr;
    HIP_OR(c, radix_sort_pairs(c->stream, txn_rank, iota, n, 32, sort_scratch, &sk, &sv));
    HIP_OR(c, gputx_kstart(c->stream, sk, n, kstart));
    HIP_OR(c, gputx_reset(c->stream, c->d_ctl));
    a.order = sv;
    a.order_rank = sk;
  }
  HIP_OR(c, hipEventRecord(c->ev[5], c->stream));
  HIP_OR(c, hipEventRecord(c->ev[1], c->stream));
  if (n) {
    hipError_t e = launch_gputx_pass(c->stream, true, (int)lanes, (int)b.max_ops, (int)wpw, (int)p.grid, strict, a,
                                     c->n_cu, &grid_used);
    if (e != hipSuccess) return launch_error(c, e);
  }
  HIP_OR(c, hipEventRecord(c->ev[2], c->stream));
  HIP_OR(c, hipEventRecord(c->ev[3], c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  Ctl h{};
  HIP_OR(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  float ms_run = 0, ms_prep = 0, ms_kernel = 0;
  HIP_OR(c, hipEventElapsedTime(&ms_run, c->ev[0], c->ev[3]));
  HIP_OR(c, hipEventElapsedTime(&ms_prep, c->ev[4], c->ev[5]));
  HIP_OR(c, hipEventElapsedTime(&ms_kernel, c->ev[1], c->ev[2]));
  std::memset(b.stats, 0, sizeof(b.stats));
  b.stats[CC_STAT_COMMITTED] = h.stats[DS_COMMITTED];
  b.stats[CC_STAT_ATTEMPTS] = h.stats[DS_ATTEMPTS];
  b.stats[CC_STAT_KERNEL_NS] = (uint64_t)((double)ms_kernel * 1e6);
  b.stats[CC_STAT_RUN_NS] = (uint64_t)((double)ms_run * 1e6);
  b.stats[CC_STAT_PREP_NS] = (uint64_t)((double)ms_prep * 1e6);
  b.stats[CC_STAT_INDEX_NS] = (uint64_t)((double)ms_index * 1e6);
  b.stats[CC_STAT_MAX_ATTEMPTS] = h.stats[DS_MAX_ATTEMPTS];
  b.stats[CC_STAT_PASSES] = n ? 1 : 0;
  b.stats[CC_STAT_GRID] = (uint64_t)grid_used;
  b.stats[CC_STAT_PACKED_STATE] = packed ? 1 : 0;
  const double ns_per_tick = 1e6 / (double)c->wallclock_khz;
  b.stats[CC_STAT_T_USEFUL_NS] = (uint64_t)((double)h.stats[DS_T_USEFUL] * ns_per_tick);
  b.stats[CC_STAT_T_WAIT_NS] = (uint64_t)((double)h.stats[DS_T_WAIT] * ns_per_tick);
  b.ran = true;
  if (n) {
    std::vector<cc_outcome> o(n);
    HIP_OR(c, hipMemcpy(o.data(), b.d_out, n * sizeof(cc_outcome), hipMemcpyDeviceToHost));
    uint64_t ksets = 0;
    for (auto &x : o)
      if (x.status == CC_COMMITTED) ksets = std::max<uint64_t>(ksets, x.serial_hi + 1);
    b.stats[CC_STAT_KSETS] = ksets;
    latency_percentiles(o, &b.stats[CC_STAT_LAT_P50_NS], &b.stats[CC_STAT_LAT_P99_NS]);
  }
  if (h.stop) return fail(c, CC_E_LIVELOCK, "CC_GPUTX: a transaction waited past the limit");
  if (h.stats[DS_COMMITTED] != n) return fail(c, CC_E_LIVELOCK, "CC_GPUTX: not every transaction ran");
  return CC_OK;
}

// The hot-row engine's plan from the per-row write counts (see find_hot_rows).
static void plan_engine(const DevOp *dops, const DevTxn *dtx, uint64_t n_txns, const std::vector<Table> &tables,
                        const std::vector<uint32_t> &cnt, Batch &b) {
  b.eng = EngineArgs{};
  b.n_eng_txns = 0;
  b.eng_gain = false;
  b.eng_part.clear();
  b.eng_desc.clear();
  const uint32_t thr = (uint32_t)std::max<uint64_t>(2, n_txns / 4096);
  // candidates: the most written rows (more than fit, to know the best row left out)
  constexpr int NC = ENG_MAX + 16;
  uint32_t cc[NC] = {}, cr[NC] = {};
  int nc = 0;
  for (uint64_t r = 0; r < cnt.size(); ++r) {
    const uint32_t c = cnt[r];
    if (c == 0 || (nc == NC && c <= cc[NC - 1])) continue;
    int i = nc < NC ? nc++ : NC - 1;
    while (i > 0 && cc[i - 1] < c) {
      cc[i] = cc[i - 1];
      cr[i] = cr[i - 1];
      --i;
    }
    cc[i] = c;
    cr[i] = (uint32_t)r;
  }
  if (nc == 0 || cc[0] < thr) return;
  uint32_t left_out = 0;  // writes of the most written row not taken
  bool full = false;
  for (int i = 0; i < nc; ++i) {
    const uint32_t r = cr[i];
    const Table *tb = nullptr;
    for (const Table &t : tables)
      if (r >= t.row_base && r < t.row_base + t.n_rows) tb = &t;
    bool take = !full && cc[i] >= thr && tb && tb->n_fields <= (uint32_t)ENG_FIELDS &&
                b.eng.n_vals + tb->n_fields <= (uint32_t)ENG_VALS;
    if (take) {
      const uint32_t k = b.eng.n_rows++;
      b.eng.row[k] = r;
      b.eng.elem0[k] = (uint32_t)(tb->elem_base + (r - tb->row_base) * tb->n_fields);
      b.eng.off[k] = b.eng.n_vals;
      b.eng.n_vals += tb->n_fields;
      full = b.eng.n_rows == (uint32_t)ENG_MAX;
    } else if (!left_out) {
      left_out = cc[i];
    }
  }
  if (b.eng.n_rows == 0) return;
  b.eng.off[b.eng.n_rows] = b.eng.n_vals;
  // a row below the candidates is written at most as often as the last candidate
  if (!left_out && nc == NC) left_out = cc[NC - 1];
  b.eng_gain = (uint64_t)left_out * 4 <= (uint64_t)cc[0];
  std::vector<uint8_t> eng_of(cnt.size(), 0);  // engine index + 1 of a row (0: not an engine row)
  for (uint32_t k = 0; k < b.eng.n_rows; ++k) eng_of[b.eng.row[k]] = (uint8_t)(k + 1);
  std::vector<uint8_t> in_eng(n_txns, 0);
  for (uint64_t t = 0; t < n_txns; ++t)
    for (uint32_t i = 0; i < dtx[t].n && !in_eng[t]; ++i) {
      const uint32_t rk = dops[dtx[t].first + i].rowk;
      in_eng[t] = (rk & WRITTEN_BIT) && eng_of[rk & ROW_MASK];
    }
  b.eng_part.reserve(n_txns);
  for (uint64_t t = 0; t < n_txns; ++t)
    if (in_eng[t]) {
      uint32_t emask = 0;  // the engine rows the transaction touches, read or written
      for (uint32_t i = 0; i < dtx[t].n; ++i) {
        const uint32_t k = eng_of[dops[dtx[t].first + i].rowk & ROW_MASK];
        if (k) emask |= 1u << (k - 1);
      }
      b.eng_part.push_back((uint32_t)t);
      b.eng_desc.push_back(EngineDesc{(uint32_t)t, dtx[t].first, dtx[t].n, emask});
    }
  b.n_eng_txns = b.eng_part.size();
  for (uint64_t t = 0; t < n_txns; ++t)
    if (!in_eng[t]) b.eng_part.push_back((uint32_t)t);
  if (b.n_eng_txns == 0) {
    b.eng = EngineArgs{};
    b.eng_part.clear();
    b.eng_desc.clear();
  }
}

// Uploads the engine's transaction order planned at submission (nothing
// without engine rows).
static hipError_t upload_engine_plan(cc_ctx *c, Batch &b) {
  if (b.n_eng_txns == 0) return hipSuccess;
  hipError_t e = hipMalloc(&b.d_part, b.eng_part.size() * sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.d_part, b.eng_part.data(), b.eng_part.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipMalloc(&b.d_eng_desc, b.eng_desc.size() * sizeof(EngineDesc));
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.d_eng_desc, b.eng_desc.data(), b.eng_desc.size() * sizeof(EngineDesc),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  b.eng_part = std::vector<uint32_t>();
  b.eng_desc = std::vector<EngineDesc>();
  return e;
}

// The batch's most written rows, counted at submission from its packed
// descriptors: write accesses (row groups that write) per global row; the
// most written row, and every row written at least a quarter as often, at
// most HOT_MAX of them, most written first (ties: lower row first).
//
// With them, the OCC hot-row engine's plan (hot_engine.h): its rows are the
// most written rows, at most ENG_MAX, each written at least
// max(2, n_txns / 4096) times, of at most ENG_FIELDS fields and ENG_VALS
// cells in all, most written first; its transactions are those that write
// one of them, listed first in eng_part (in batch order), the others after
// them.  eng_gain holds when every row left out is written at most a quarter
// as often as the most written row: otherwise the rest of the batch is about
// as contended as the engine's share, and the engine's serial pass gains
// nothing.
void find_hot_rows(const DevOp *dops, uint64_t n_ops, const DevTxn *dtx, uint64_t n_txns,
                   const std::vector<Table> &tables, uint64_t total_rows, Batch &b) {
  std::vector<uint32_t> cnt(std::max<uint64_t>(total_rows, 1), 0u);
  for (uint64_t i = 0; i < n_ops; ++i) {
    const uint32_t rk = dops[i].rowk;
    if (!(rk & FOLLOWER_BIT) && (rk & WRITTEN_BIT)) ++cnt[rk & ROW_MASK];
  }
  if (b.scheme == CC_OCC) plan_engine(dops, dtx, n_txns, tables, cnt, b);
  uint32_t top = 0;
  for (uint32_t c : cnt) top = std::max(top, c);
  b.hot_known = true;
  b.hot_writes = top;
  b.n_hot = 0;
  if (top == 0) return;
  const uint32_t thr = std::max<uint32_t>(1u, (top + 3) / 4);
  uint32_t best_c[HOT_MAX] = {}, best_r[HOT_MAX] = {};
  uint32_t n = 0;
  for (uint64_t r = 0; r < total_rows; ++r) {
    const uint32_t c = cnt[r];
    if (c < thr || (n == (uint32_t)HOT_MAX && c <= best_c[HOT_MAX - 1])) continue;
    uint32_t i = n < (uint32_t)HOT_MAX ? n++ : (uint32_t)HOT_MAX - 1;
    while (i > 0 && best_c[i - 1] < c) {
      best_c[i] = best_c[i - 1];
      best_r[i] = best_r[i - 1];
      --i;
    }
    best_c[i] = c;
    best_r[i] = (uint32_t)r;
  }
  for (uint32_t i = 0; i < n; ++i) b.hot_rows[i] = best_r[i];
  b.n_hot = n;
}

// Run parameters against the scheme, before anything touches the device
// (cc_check_run_params and cc_run).  c may be NULL (no message kept).
cc_status check_run_params(cc_ctx *c, int scheme, const cc_run_params &p) {
  if (scheme < 0 || scheme >= CC_N_SCHEMES) return fail(c, CC_E_INVAL, "unknown scheme");
  if (p.mode != CC_MODE_PLAIN && p.mode != CC_MODE_EPOCH && p.mode != CC_MODE_SERVE)
    return fail(c, CC_E_INVAL, "unknown mode");
  const uint32_t lanes = p.lanes_per_txn;
  if (lanes != 0 && lanes != 1 && lanes != 4 && lanes != 16 && lanes != 64)
    return fail(c, CC_E_INVAL, "lanes_per_txn must be 1, 4, 16 or 64");
  if (p.waves_per_wg > 16) return fail(c, CC_E_INVAL, "waves_per_wg must be 1..16");
  if (p.flags & ~(CC_RUN_STRICT_FENCES | CC_RUN_EAGER_INSTALL | CC_RUN_WAIT_UNLOCK | CC_RUN_PRECHECK |
                  CC_RUN_NO_PRECHECK | CC_RUN_INDEX_TREE | CC_RUN_LATCH | CC_RUN_SHARED_READS | CC_RUN_HOT_LAST |
                  CC_RUN_NO_HOT_LAST | CC_RUN_WAIT_BLOCKER | CC_RUN_HOT_ENGINE | CC_RUN_NO_HOT_ENGINE))
    return fail(c, CC_E_INVAL, "unknown run flag");
  if ((p.flags & CC_RUN_SHARED_READS) && scheme != CC_GACCO)
    return fail(c, CC_E_INVAL, "CC_RUN_SHARED_READS is a CC_GACCO option");
  if (p.wait_limit_us && scheme != CC_GACCO && scheme != CC_GPUTX)
    return fail(c, CC_E_INVAL, "wait_limit_us applies to CC_GACCO and CC_GPUTX only");
  if (p.flags & CC_RUN_WAIT_UNLOCK)
    // Switched off: two teams of one wavefront that block each other both see
    // the row free on their next loop iteration (each attempt releases its
    // locks before returning) and retry together, so in the final
    // single-wavefront pass, which never defers, they can conflict forever.
    return fail(c, CC_E_INVAL, "CC_RUN_WAIT_UNLOCK is disabled (same-wavefront retries can livelock)");
  if (scheme == CC_GACCO) {
    if (p.mode != CC_MODE_PLAIN)
      return fail(c, CC_E_INVAL,
                  "CC_GACCO runs in CC_MODE_PLAIN only: it never aborts, so epochs have nothing to retry, and it "
                  "orders the whole batch before running it");
    if (p.flags & ~(CC_RUN_STRICT_FENCES | CC_RUN_INDEX_TREE | CC_RUN_SHARED_READS))
      return fail(c, CC_E_INVAL, "CC_GACCO accepts only CC_RUN_STRICT_FENCES, CC_RUN_INDEX_TREE and CC_RUN_SHARED_READS");
    return CC_OK;
  }
  if (scheme == CC_GPUTX) {
    if (p.mode != CC_MODE_PLAIN)
      return fail(c, CC_E_INVAL, "CC_GPUTX runs in CC_MODE_PLAIN only: it orders the whole batch before running it");
    if (p.flags & ~(CC_RUN_STRICT_FENCES | CC_RUN_INDEX_TREE))
      return fail(c, CC_E_INVAL, "CC_GPUTX accepts only CC_RUN_STRICT_FENCES and CC_RUN_INDEX_TREE");
    return CC_OK;
  }
  const uint32_t pre = CC_RUN_PRECHECK | CC_RUN_NO_PRECHECK;
  if ((p.flags & pre) == pre) return fail(c, CC_E_INVAL, "CC_RUN_PRECHECK and CC_RUN_NO_PRECHECK exclude each other");
  if ((p.flags & pre) && scheme != CC_OCC && scheme != CC_TICTOC && scheme != CC_TO && scheme != CC_MVCC)
    return fail(c, CC_E_INVAL, "the pre-check round exists for CC_OCC, CC_TICTOC, CC_TO and CC_MVCC only");
  if ((p.flags & CC_RUN_EAGER_INSTALL) && scheme != CC_OCC)
    return fail(c, CC_E_INVAL, "CC_RUN_EAGER_INSTALL is a CC_OCC option");
  const uint32_t hot = CC_RUN_HOT_LAST | CC_RUN_NO_HOT_LAST;
  if ((p.flags & hot) == hot) return fail(c, CC_E_INVAL, "CC_RUN_HOT_LAST and CC_RUN_NO_HOT_LAST exclude each other");
  if ((p.flags & hot) && scheme != CC_OCC) return fail(c, CC_E_INVAL, "CC_RUN_HOT_LAST is a CC_OCC option");
  if ((p.flags & CC_RUN_WAIT_BLOCKER) && scheme != CC_OCC && scheme != CC_TICTOC)
    return fail(c, CC_E_INVAL, "CC_RUN_WAIT_BLOCKER is a CC_OCC and CC_TICTOC option");
  const uint32_t eng = CC_RUN_HOT_ENGINE | CC_RUN_NO_HOT_ENGINE;
  if ((p.flags & eng) == eng) return fail(c, CC_E_INVAL, "CC_RUN_HOT_ENGINE and CC_RUN_NO_HOT_ENGINE exclude each other");
  if ((p.flags & eng) && scheme != CC_OCC) return fail(c, CC_E_INVAL, "CC_RUN_HOT_ENGINE is a CC_OCC option");
  if ((p.flags & CC_RUN_HOT_ENGINE) && p.mode != CC_MODE_PLAIN)
    return fail(c, CC_E_INVAL, "CC_RUN_HOT_ENGINE runs in CC_MODE_PLAIN only");
  if ((p.flags & CC_RUN_HOT_ENGINE) && (p.flags & CC_RUN_LATCH))
    return fail(c, CC_E_INVAL, "CC_RUN_HOT_ENGINE does not take CC_RUN_LATCH");
  return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_check_batch(uint32_t n_tables, const uint64_t *n_rows, const uint32_t *n_fields, const cc_txn *txns,
                         uint64_t n_txns, const cc_op *ops, uint64_t n_ops, int scheme) {
  if (n_tables > CC_MAX_TABLES || (n_tables && (!n_rows || !n_fields))) return CC_E_INVAL;
  if (scheme < 0 || scheme >= CC_N_SCHEMES) return CC_E_INVAL;
  uint64_t rows = 0, cells = 0;
  for (uint32_t t = 0; t < n_tables; ++t) {
    if (n_rows[t] == 0 || n_fields[t] == 0 || n_fields[t] > 256) return CC_E_INVAL;
    rows += n_rows[t];
    cells += n_rows[t] * n_fields[t];
  }
  if (rows > CC_MAX_TOTAL_ROWS || cells > CC_MAX_TOTAL_CELLS) return CC_E_RANGE;
  bool ordered = true;
  const cc_status st = validate_and_pack(nullptr, layout_tables(n_tables, n_rows, n_fields), txns, n_txns, ops, n_ops,
                                         nullptr, nullptr, nullptr, nullptr, &ordered);
  if (st == CC_OK && (scheme == CC_GACCO || scheme == CC_GPUTX) && !ordered) return CC_E_INVAL;
  return st;
}

// Device buffers of a batch: descriptors, outcomes, read values, pending
// list, and the scheme's extras.  All or nothing.
static hipError_t alloc_batch(Batch &b, int scheme, bool keyed) {
  const bool ordered_scheme = scheme == CC_GACCO || scheme == CC_GPUTX;
  const uint64_t n_ops = b.n_ops, n_txns = b.n_txns;
  auto alloc = [&](void **p, size_t bytes) -> hipError_t { return hipMalloc(p, bytes ? bytes : 16); };
  hipError_t e;
  if ((e = alloc((void **)&b.d_ops, n_ops * sizeof(DevOp))) != hipSuccess ||
      (e = alloc((void **)&b.d_txns, n_txns * sizeof(DevTxn))) != hipSuccess ||
      (e = alloc((void **)&b.d_out, n_txns * sizeof(DevOutcome))) != hipSuccess ||
      (e = alloc((void **)&b.d_reads, n_ops * sizeof(int64_t))) != hipSuccess ||
      (e = alloc((void **)&b.d_list, n_txns * sizeof(uint32_t))) != hipSuccess ||
      (ordered_scheme && (e = alloc((void **)&b.d_rank, n_ops * sizeof(uint32_t))) != hipSuccess) ||
      (ordered_scheme &&
       (e = alloc((void **)&b.d_gscratch, gacco_scratch_words(n_ops) * sizeof(uint32_t))) != hipSuccess) ||
      (scheme == CC_GPUTX &&
       (e = alloc((void **)&b.d_tscratch, gputx_scratch_words(n_txns) * sizeof(uint32_t))) != hipSuccess) ||
      (keyed && (e = alloc((void **)&b.d_opkeys, n_ops * sizeof(int64_t))) != hipSuccess) ||
      (keyed && (e = alloc((void **)&b.d_meta, n_ops * sizeof(uint32_t))) != hipSuccess) ||
      (keyed && (e = alloc((void **)&b.d_rows, n_ops * sizeof(uint32_t))) != hipSuccess)) {
    free_batch(b);
    return e;
  }
  return hipSuccess;
}

// True if [p, p + bytes) lies inside one allocation of the context's device.
static bool device_range(const cc_ctx *c, const void *p, uint64_t bytes) {
  if (bytes == 0) return true;
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeDevice || at.device != c->device) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const uintptr_t lo = (uintptr_t)base, q = (uintptr_t)p;
  return q >= lo && bytes <= size && q - lo <= size - bytes;
}

static const char *ingest_message(uint32_t m) {
  switch (m) {
    case INGEST_MSG_RESERVED: return "cc_txn.reserved must be 0";
    case INGEST_MSG_TOO_MANY: return "transaction has too many ops";
    case INGEST_MSG_OP_RANGE: return "op range outside ops";
    case INGEST_MSG_SHARED: return "transactions share operations";
    case INGEST_MSG_TABLE: return "op table out of range";
    case INGEST_MSG_KEYED_ROW: return "an op on an indexed table names its row by key; row must be 0";
    case INGEST_MSG_ROW_FIELD: return "op row/field out of range";
    case INGEST_MSG_KIND: return "unknown op kind";
    case INGEST_MSG_SLOT_SRC: return "WRITE_SLOT source is not an earlier op";
    case INGEST_MSG_DUP_FIELD: return "field repeated within a txn";
    case INGEST_MSG_DUP_ROW: return "row accessed twice (non-adjacent) within a txn";
    default: return "malformed batch";
  }
}

static cc_status submit_impl(cc_ctx *c, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                             const int64_t *op_keys, int scheme, int on_device, uint64_t *batch_id) {
  if (!c || !batch_id) return CC_E_INVAL;
  *batch_id = 0;
  if (scheme < 0 || scheme >= CC_N_SCHEMES) return fail(c, CC_E_INVAL, "unknown scheme");
  if (!c->frozen) return fail(c, CC_E_STATE, "load the tables before submitting a batch");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  std::vector<bool> indexed(c->tables.size(), false);
  for (size_t t = 0; t < c->indexes.size() && t < indexed.size(); ++t) indexed[t] = c->indexes[t].keys != nullptr;
  const bool ordered_scheme = scheme == CC_GACCO || scheme == CC_GPUTX;
  Batch b;
  b.scheme = scheme;
  b.n_txns = n_txns;
  b.n_ops = n_ops;

  if (on_device) {
    // the caller's arrays are in device memory: validate and pack them there
    if ((n_txns && !txns) || (n_ops && !ops)) return fail(c, CC_E_INVAL, "null array");
    if (n_txns > 0xFFFFFFFFull || n_ops > 0xFFFFFFFFull) return fail(c, CC_E_RANGE, "batch too large");
    if (!device_range(c, txns, n_txns * sizeof(cc_txn)) || !device_range(c, ops, n_ops * sizeof(cc_op)) ||
        (op_keys && !device_range(c, op_keys, n_ops * sizeof(int64_t))))
      return fail(c, CC_E_INVAL, "on_device arrays must lie in device memory of the context's device");
    bool any_index = false;
    for (bool x : indexed) any_index |= x;
    const bool maybe_keyed = op_keys && any_index;
    hipError_t e = alloc_batch(b, scheme, maybe_keyed);
    if (e != hipSuccess) return hip_fail(c, e, "batch allocation");
    if (!c->d_ingest && (e = hipMalloc(&c->d_ingest, INGEST_N * sizeof(uint64_t))) != hipSuccess) {
      free_batch(b);
      return hip_fail(c, e, "ingest buffer allocation");
    }
    IngestArgs ia{};
    ia.txns = txns;
    ia.ops = ops;
    ia.op_keys = maybe_keyed ? op_keys : nullptr;
    ia.n_txns = n_txns;
    ia.n_ops = n_ops;
    ia.n_tables = (uint32_t)c->tables.size();
    for (uint32_t t = 0; t < ia.n_tables; ++t) {
      const Table &tb = c->tables[t];
      ia.tab[t] = IngestTable{tb.n_rows, tb.row_base, tb.elem_base, tb.n_fields, (uint32_t)(indexed[t] ? 1 : 0)};
    }
    ia.dops = b.d_ops;
    ia.dtx = b.d_txns;
    ia.owner = (uint32_t *)b.d_reads;  // n_ops x 8 bytes, cleared below before any run
    ia.meta = maybe_keyed ? b.d_meta : nullptr;
    ia.rows0 = maybe_keyed ? b.d_rows : nullptr;
    ia.out = c->d_ingest;
    uint64_t res[INGEST_N] = {};
    e = launch_ingest(c->stream, ia);
    if (e == hipSuccess && maybe_keyed && n_ops)
      e = hipMemcpyAsync(b.d_opkeys, op_keys, n_ops * sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && n_ops) e = hipMemsetAsync(b.d_reads, 0, n_ops * sizeof(int64_t), c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(res, c->d_ingest, sizeof res, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(c, e, "batch ingest");
    }
    if (res[INGEST_ERR] != ~0ull) {
      free_batch(b);
      const uint64_t w = res[INGEST_ERR];
      const cc_status code = -(cc_status)(w & 15u);
      return fail(c, code, std::string(ingest_message((uint32_t)((w >> 4) & 0xFFFu))) + " (transaction " +
                               std::to_string(w >> 16) + ")");
    }
    if (ordered_scheme && res[INGEST_UNORDERED]) {
      free_batch(b);
      return fail(c, CC_E_INVAL,
                  "CC_GACCO and CC_GPUTX need each transaction's ops after the previous transaction's (first_op "
                  "nondecreasing)");
    }
    b.max_ops = (uint32_t)res[INGEST_MAX_OPS];
    b.has_slot = res[INGEST_HAS_SLOT] != 0;
    b.keyed = res[INGEST_KEYED] != 0;
    if (maybe_keyed && !b.keyed) {
      (void)hipFree(b.d_opkeys);
      (void)hipFree(b.d_meta);
      (void)hipFree(b.d_rows);
      b.d_opkeys = nullptr;
      b.d_meta = nullptr;
      b.d_rows = nullptr;
    }
    if (!b.keyed) {
      // the packed descriptors come back once, to count the rows' writes
      std::vector<DevOp> hd(n_ops);
      std::vector<DevTxn> ht(n_txns);
      if (n_ops && (e = hipMemcpy(hd.data(), b.d_ops, n_ops * sizeof(DevOp), hipMemcpyDeviceToHost)) != hipSuccess) {
        free_batch(b);
        return hip_fail(c, e, "batch descriptors");
      }
      if (n_txns && (e = hipMemcpy(ht.data(), b.d_txns, n_txns * sizeof(DevTxn), hipMemcpyDeviceToHost)) != hipSuccess) {
        free_batch(b);
        return hip_fail(c, e, "batch descriptors");
      }
      find_hot_rows(hd.data(), n_ops, ht.data(), n_txns, c->tables, c->total_rows, b);
      if ((e = upload_engine_plan(c, b)) != hipSuccess) {
        free_batch(b);
        return hip_fail(c, e, "engine plan upload");
      }
    }
    const uint64_t id = c->next_batch++;
    c->batches[id] = b;
    *batch_id = id;
    return CC_OK;
  }

  std::vector<DevOp> dops;
  std::vector<DevTxn> dtx;
  uint32_t max_ops = 0;
  bool has_slot = false, ordered = true;
  cc_status st = validate_and_pack(c, c->tables, txns, n_txns, ops, n_ops, &dops, &dtx, &max_ops, &has_slot, &ordered,
                                   op_keys, op_keys ? &indexed : nullptr);
  if (st) return st;
  if (ordered_scheme && !ordered)
    return fail(c, CC_E_INVAL,
                "CC_GACCO and CC_GPUTX need each transaction's ops after the previous transaction's (first_op nondecreasing)");
  // keyed ops of the transactions (ops no transaction refers to are never looked up)
  std::vector<uint32_t> meta;
  std::vector<uint32_t> rows0;
  bool keyed = false;
  if (op_keys) {
    meta.assign(n_ops, 0u);
    rows0.assign(n_ops, 0u);
    for (uint64_t i = 0; i < n_ops; ++i) rows0[i] = ops[i].row;
    for (uint64_t t = 0; t < n_txns; ++t)
      for (uint32_t i = 0; i < txns[t].n_ops; ++i) {
        const uint64_t k = txns[t].first_op + i;
        if (indexed[ops[k].table]) {
          meta[k] = META_KEYED | ((uint32_t)ops[k].table << 16) | ops[k].field;
          keyed = true;
        }
      }
  }
  b.max_ops = max_ops;
  b.has_slot = has_slot;
  b.keyed = keyed;
  // keyed ops learn their rows only when the index is searched, at the run
  if (!keyed) find_hot_rows(dops.data(), n_ops, dtx.data(), n_txns, c->tables, c->total_rows, b);
  hipError_t e = alloc_batch(b, scheme, keyed);
  if (e != hipSuccess) return hip_fail(c, e, "batch allocation");
  auto copy_in = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    if (n_ops) r = hipMemcpyAsync(b.d_ops, dops.data(), n_ops * sizeof(DevOp), hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess && n_txns)
      r = hipMemcpyAsync(b.d_txns, dtx.data(), n_txns * sizeof(DevTxn), hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess && n_ops) r = hipMemsetAsync(b.d_reads, 0, n_ops * sizeof(int64_t), c->stream);
    if (r == hipSuccess && keyed)
      r = hipMemcpyAsync(b.d_opkeys, op_keys, n_ops * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess && keyed)
      r = hipMemcpyAsync(b.d_meta, meta.data(), n_ops * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess && keyed)
      r = hipMemcpyAsync(b.d_rows, rows0.data(), n_ops * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    return r;
  };
  if ((e = copy_in()) != hipSuccess || (e = upload_engine_plan(c, b)) != hipSuccess) {
    free_batch(b);
    return hip_fail(c, e, "batch upload");
  }
  const uint64_t id = c->next_batch++;
  c->batches[id] = b;
  *batch_id = id;
  return CC_OK;
}

cc_status cc_submit_batch(cc_ctx *c, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                          int scheme, int on_device, uint64_t *batch_id) {
  return submit_impl(c, txns, n_txns, ops, n_ops, nullptr, scheme, on_device, batch_id);
}

cc_status cc_submit_batch_keyed(cc_ctx *c, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops,
                                const int64_t *op_keys, int scheme, int on_device, uint64_t *batch_id) {
  if (!op_keys && n_ops) return fail(c, CC_E_INVAL, "op_keys is NULL");
  return submit_impl(c, txns, n_txns, ops, n_ops, op_keys, scheme, on_device, batch_id);
}

cc_status cc_create_index(cc_ctx *c, uint32_t tid, const int64_t *keys, uint64_t n) {
  if (!c || (!keys && n)) return CC_E_INVAL;
  if (tid >= c->tables.size()) return fail(c, CC_E_RANGE, "unknown table");
  if (n != c->tables[tid].n_rows) return fail(c, CC_E_INVAL, "one key per row of the table");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  cc_status st = freeze(c);
  if (st) return st;
  for (auto &kv : c->batches)
    if (kv.second.keyed) return fail(c, CC_E_STATE, "release the keyed batches before changing an index");
  // sort (key, row) on the host: index construction is load-time work
  std::vector<std::pair<int64_t, uint32_t>> kr(n);
  for (uint64_t i = 0; i < n; ++i) {
    if (keys[i] == INT64_MAX) return fail(c, CC_E_INVAL, "INT64_MAX is reserved (index padding)");
    kr[i] = {keys[i], (uint32_t)i};
  }
  std::sort(kr.begin(), kr.end());
  for (uint64_t i = 1; i < n; ++i)
    if (kr[i].first == kr[i - 1].first) return fail(c, CC_E_INVAL, "index keys must be distinct");
  auto pad16 = [](uint64_t m) { return (m + 15) / 16 * 16; };
  std::vector<int64_t> level0(pad16(std::max<uint64_t>(n, 1)), INT64_MAX);
  std::vector<uint32_t> rows(std::max<uint64_t>(n, 1), 0u);
  for (uint64_t i = 0; i < n; ++i) {
    level0[i] = kr[i].first;
    rows[i] = kr[i].second;
  }
  // upper levels: the largest key of each 16-key node of the level below
  std::vector<int64_t> tree;
  IndexDesc d{};
  d.n = n;
  std::vector<int64_t> cur = level0;
  uint64_t real = n;  // entries of `cur` that are keys (the rest is padding)
  uint32_t levels = 0;
  while (cur.size() > 16) {
    if (levels >= INDEX_MAX_LEVELS) return fail(c, CC_E_RANGE, "index too large");
    const uint64_t nodes = (real + 15) / 16;
    std::vector<int64_t> up(pad16(nodes), INT64_MAX);
    for (uint64_t j = 0; j < nodes; ++j) up[j] = cur[std::min(j * 16 + 15, real - 1)];
    real = nodes;
    ++levels;
    d.level_off[levels] = tree.size();
    tree.insert(tree.end(), up.begin(), up.end());
    cur.swap(up);
  }
  d.levels = levels;
  const Table &t = c->tables[tid];
  d.row_base = t.row_base;
  d.elem_base = t.elem_base;
  d.n_fields = t.n_fields;
  // Build the new index in full before touching the old one: on any failure
  // the table keeps its previous index (or none), on the host and on the
  // device alike.
  DevIndex nx{};
  auto drop = [](DevIndex &x) {
    if (x.keys) (void)hipFree(x.keys);
    if (x.rows) (void)hipFree(x.rows);
    if (x.tree) (void)hipFree(x.tree);
    x = DevIndex{};
  };
  if (!c->d_idx) HIP_OR(c, hipMalloc(&c->d_idx, CC_MAX_TABLES * sizeof(IndexDesc)));
  hipError_t e = hipMalloc(&nx.keys, level0.size() * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&nx.rows, rows.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&nx.tree, std::max<size_t>(tree.size(), 1) * sizeof(int64_t));
  if (e == hipSuccess)
    e = hipMemcpyAsync(nx.keys, level0.data(), level0.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(nx.rows, rows.data(), rows.size() * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !tree.empty())
    e = hipMemcpyAsync(nx.tree, tree.data(), tree.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    drop(nx);
    return hip_fail(c, e, "index upload");
  }
  d.keys = nx.keys;
  d.rows = nx.rows;
  d.tree = nx.tree;
  nx.desc = d;
  std::vector<IndexDesc> all(CC_MAX_TABLES, IndexDesc{});
  for (size_t i = 0; i < c->indexes.size(); ++i) all[i] = c->indexes[i].desc;
  all[tid] = d;
  e = hipMemcpyAsync(c->d_idx, all.data(), all.size() * sizeof(IndexDesc), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    // the device table may be partly written: put the old descriptors back
    // (best effort) and keep the old index
    for (size_t i = 0; i < c->indexes.size(); ++i) all[i] = c->indexes[i].desc;
    if (tid >= c->indexes.size()) all[tid] = IndexDesc{};
    (void)hipMemcpy(c->d_idx, all.data(), all.size() * sizeof(IndexDesc), hipMemcpyHostToDevice);
    drop(nx);
    return hip_fail(c, e, "index descriptor upload");
  }
  if (c->indexes.size() < c->tables.size()) c->indexes.resize(c->tables.size());
  drop(c->indexes[tid]);
  c->indexes[tid] = nx;
  return CC_OK;
}

cc_status cc_engine_plan(cc_ctx *c, uint64_t batch_id, uint32_t *rows, uint32_t *n_rows, uint64_t *n_txns,
                         int *by_default) {
  if (!c || !rows || !n_rows || !n_txns || !by_default) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  const Batch &b = it->second;
  static_assert(CC_ENGINE_MAX_ROWS == ENG_MAX, "engine rows");
  for (uint32_t i = 0; i < (uint32_t)ENG_MAX; ++i) rows[i] = i < b.eng.n_rows ? b.eng.row[i] : 0u;
  *n_rows = b.n_eng_txns ? b.eng.n_rows : 0;
  *n_txns = b.n_eng_txns;
  *by_default = b.n_eng_txns && b.eng_gain ? 1 : 0;
  return CC_OK;
}

cc_status cc_fetch_rows(cc_ctx *c, uint64_t batch_id, uint32_t *rows) {
  if (!c || !rows) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  Batch &b = it->second;
  if (!b.keyed) return fail(c, CC_E_STATE, "the batch has no keyed operations");
  if (!b.ran) return fail(c, CC_E_STATE, "batch has not been run");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  if (b.n_ops) HIP_OR(c, hipMemcpy(rows, b.d_rows, b.n_ops * sizeof(uint32_t), hipMemcpyDeviceToHost));
  return CC_OK;
}

cc_status cc_check_run_params(int scheme, const cc_run_params *pp) {
  return check_run_params(nullptr, scheme, pp ? *pp : cc_run_params{});
}

}  // extern "C"

// One run of a batch whose parameters have been checked (cc_run, and
// cc_run_static with a batch that lives in the static scratch).  host_stats:
// copy the outcomes back for the latency percentiles.
static cc_status run_batch(cc_ctx *c, Batch &b, const cc_run_params &p, bool host_stats) {
  if (p.mode == CC_MODE_SERVE && b.n_txns && !b.d_arrival)
    return fail(c, CC_E_STATE, "CC_MODE_SERVE needs cc_set_arrivals first");
  // contention of the batch: the share of transactions that write its most
  // written row (unknown: treated as contended)
  const double hot_share = b.hot_known && b.n_txns ? (double)b.hot_writes / (double)b.n_txns : 1.0;
  const bool no_hot_row = hot_share < 0.001, contended = hot_share >= 0.02;
  uint32_t lanes = p.lanes_per_txn;
  uint32_t wpw = p.waves_per_wg;
  if (lanes == 0) {
    if (no_hot_row && b.max_ops <= 64 && b.scheme != CC_GACCO && b.scheme != CC_GPUTX) {
      // nothing to wait for: 4 lanes per transaction, 4 wavefronts per
      // workgroup (4096 transactions in flight at one workgroup per CU)
      lanes = 4;
      if (wpw == 0) wpw = 4;
    } else {
      lanes = 1;
      while (lanes < 64 && lanes < b.max_ops) lanes *= 4;
    }
  }
  if (wpw == 0) wpw = 1;
  // the hot-row engine has variants up to 4 ops per lane; unless the caller
  // chose, it runs one transaction per wavefront (64 lanes): its waiting teams
  // then poll without waiting for other teams' round trips
  const uint32_t eng_lanes = p.lanes_per_txn ? lanes : 64;
  const bool eng_fits = (b.max_ops + eng_lanes - 1) / eng_lanes <= 4;
  if ((p.flags & CC_RUN_HOT_ENGINE) && !eng_fits)
    return fail(c, CC_E_INVAL, "CC_RUN_HOT_ENGINE needs at most 4 ops per lane");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  if (b.scheme == CC_GACCO) return run_gacco(c, b, p, lanes, wpw);
  if (b.scheme == CC_GPUTX) return run_gputx(c, b, p, lanes, wpw);

  RunArgs a{};
  a.ops = b.d_ops;
  a.txns = b.d_txns;
  a.n_txns = b.n_txns;
  a.data = c->d_data;
  a.words = c->d_words;
  if (b.scheme == CC_MVCC && !c->d_aux) {
    HIP_OR(c, hipMalloc(&c->d_aux, std::max<uint64_t>(c->total_rows, 1) * sizeof(uint64_t)));
  }
  a.aux = c->d_aux;
  if (b.scheme == CC_MVCC) {
    // the version arena: one slot per op of the batch, or, when serving with
    // a cap, hbm_cap_bytes / 32 slots, reused as a ring; at least 1024 slots,
    // more than one transaction's writes (256), so that no commit's slots wrap
    // onto each other
    const uint64_t slots = (p.mode == CC_MODE_SERVE && p.hbm_cap_bytes)
                               ? std::max<uint64_t>(p.hbm_cap_bytes / 32, 1024)
                               : std::max<uint64_t>(b.n_ops, 1024);
    if (!b.d_nodes || b.node_slots != slots) {
      if (b.d_nodes) (void)hipFree(b.d_nodes);
      b.d_nodes = nullptr;
      b.node_slots = 0;
      if (b.epoch_graph) {
        // a captured epoch holds the old arena's address
        (void)hipGraphExecDestroy(b.epoch_graph);
        b.epoch_graph = nullptr;
      }
      const uint64_t bytes = 32 + slots * 4 * sizeof(uint64_t);
      HIP_OR(c, hipMalloc(&b.d_nodes, bytes));
      HIP_OR(c, hipMemsetAsync(b.d_nodes, 0, bytes, c->stream));  // tags 0 (lap 0), ring counter 0
      b.node_slots = slots;
    }
  }
  a.nodes = b.d_nodes ? b.d_nodes + 4 : nullptr;
  a.node_ring = b.d_nodes;
  a.n_nodes = b.node_slots;
  // a slot for every op: op i keeps slot i and no slot is reused in the run
  a.node_reuse = b.node_slots < b.n_ops ? 1u : 0u;
  a.out = b.d_out;
  a.reads = b.d_reads;
  a.ctl = c->d_ctl;
  a.max_attempts = p.max_attempts ? p.max_attempts : (1ull << 24);
  const uint64_t backoff_ns = p.backoff_ns ? p.backoff_ns : 200;
  a.backoff_ticks = (uint32_t)std::max<uint64_t>(1, backoff_ns * c->wallclock_khz / 1000000ull);
  a.ns_per_tick_q16 = (uint32_t)((1000000ull << 16) / c->wallclock_khz);
  a.has_slot = b.has_slot ? 1u : 0u;
  a.eager_install = (p.flags & CC_RUN_EAGER_INSTALL) ? 1u : 0u;
  a.precheck = (p.flags & CC_RUN_PRECHECK) ? 2u : ((p.flags & CC_RUN_NO_PRECHECK) ? 0u : (contended ? 1u : 0u));
  a.hot0 = b.n_hot ? b.hot_rows[0] : ~0u;
  a.wait_blocker = (p.flags & CC_RUN_WAIT_BLOCKER) ? 1u : 0u;
  a.poll_ticks = 2 * a.backoff_ticks;
  a.jitter_ticks = 2 * a.backoff_ticks;
  a.wait_max_ticks = 256ull * a.backoff_ticks;
  a.n_late = 0;
  if (b.scheme == CC_OCC && (p.flags & CC_RUN_HOT_LAST) && b.hot_known) {
    a.n_late = b.n_hot;
    for (uint32_t i = 0; i < b.n_hot; ++i) a.late[i] = b.hot_rows[i];
  }
  a.wd_wait_limit = 64;
  if (p.flags & CC_RUN_LATCH) {
    if (!c->d_latch) {
      // latches are free between critical sections, so they are cleared once
      HIP_OR(c, hipMalloc(&c->d_latch, std::max<uint64_t>(c->total_rows, 1) * sizeof(uint32_t)));
      HIP_OR(c, hipMemsetAsync(c->d_latch, 0, std::max<uint64_t>(c->total_rows, 1) * sizeof(uint32_t), c->stream));
    }
    a.latch = c->d_latch;
  }

  const uint32_t defer = p.defer_after ? p.defer_after : (p.mode == CC_MODE_SERVE ? 256 : 16);
  a.pass = 0;
  a.list = nullptr;
  if (p.mode == CC_MODE_SERVE) {
    a.arrival = b.d_arrival;
    a.budget_cap = p.hbm_cap_bytes;
    a.bytes_per_op = CC_SERVE_BYTES_PER_OP;
  }

  HIP_OR(c, hipEventRecord(c->ev[0], c->stream));
  HIP_OR(c, launch_init(c->stream, c->d_words, c->total_rows, c->d_aux, b.scheme == CC_MVCC ? c->total_rows : 0,
                        b.d_out, b.n_txns, c->d_ctl, p.ts_start));
  float ms_index = 0;
  if (b.keyed) {
    cc_status st = resolve_keys(c, b, p, &ms_index);
    if (st) return st;
  }
  Ctl h{};
  double kernel_ms = 0, engine_ms = 0;
  uint64_t engine_txns = 0;
  uint32_t passes = 0, epochs = 0;
  int first_grid = 0;
  bool epoch_limit = false;
  const bool strict = (p.flags & CC_RUN_STRICT_FENCES) != 0;
  const bool latch = (p.flags & CC_RUN_LATCH) != 0;

  // Plain passes over the pending transactions: each pass runs 8x fewer
  // workgroups than the last, down to a single wavefront that never defers,
  // so every transaction eventually runs without concurrency.
  auto plain_passes = [&](int grid, uint32_t waves, bool first_is_all) -> cc_status {
    bool all = first_is_all;
    for (;;) {
      if (!all) {
        HIP_OR(c, launch_compact(c->stream, b.d_out, b.n_txns, a.max_attempts, b.d_list, c->d_ctl));
        HIP_OR(c, hipMemcpyAsync(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
        HIP_OR(c, hipStreamSynchronize(c->stream));
        a.list = b.d_list;
        a.n_txns = h.pending_n;
        a.pass = 1;  // attempt counts continue from the outcome records
        a.n_from_ctl = 0;
        a.arrival = nullptr;  // deferred transactions have all arrived
        a.budget_cap = 0;
      }
      const bool last = grid == 1 && waves == 1;
      a.defer_after = last ? 0u : defer;
      HIP_OR(c, hipEventRecord(c->ev[1], c->stream));
      int grid_used = 0;
      hipError_t e = launch_txn(c->stream, b.scheme, (int)lanes, (int)b.max_ops, (int)waves, grid, strict, latch, a,
                                c->n_cu, &grid_used);
      if (e != hipSuccess) return launch_error(c, e);
      HIP_OR(c, hipEventRecord(c->ev[2], c->stream));
      HIP_OR(c, hipStreamSynchronize(c->stream));
      float ms = 0;
      HIP_OR(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
      kernel_ms += ms;
      if (first_grid == 0) first_grid = grid_used;
      ++passes;
      all = false;
      HIP_OR(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
      // a stuck latch stopped the run (reported below)
      if (h.stats[DS_COMMITTED] + h.stats[DS_GAVE_UP] >= b.n_txns || last || h.stop) return CC_OK;
      grid = std::max(1, grid_used / 8);
      if (grid == 1) waves = 1;
    }
  };

  if (b.n_txns && p.mode == CC_MODE_EPOCH) {
    // Epochs: every pending transaction gets defer_after (default 1) attempts,
    // aborted ones wait for the next epoch.  One epoch = [reset claim counter,
    // list the pending transactions, persistent transaction kernel over that
    // list]; EPOCHS_PER_GRAPH epochs are captured once as a hipGraph and the
    // graph is replayed until nothing is pending.  The kernel reads the
    // pending count from the control block, so the graph's arguments are fixed.
    // A replay that commits almost nothing (symmetric conflicts repeating
    // epoch after epoch) hands the rest to the plain passes, which always
    // finish.
    constexpr uint32_t EPOCHS_PER_GRAPH = 4;
    const uint32_t max_epochs = p.max_epochs ? p.max_epochs : (1u << 20);
    a.defer_after = p.defer_after ? p.defer_after : 1;
    a.pass = 1;
    a.list = b.d_list;
    a.n_from_ctl = 1;
    const uint64_t key[4] = {(uint64_t)lanes | ((uint64_t)wpw << 8) | ((uint64_t)p.grid << 16),
                             (uint64_t)p.flags | ((uint64_t)a.defer_after << 32), a.max_attempts,
                             (uint64_t)a.backoff_ticks | ((uint64_t)p.ts_start << 32)};
    if (!b.epoch_graph || std::memcmp(key, b.epoch_key, sizeof key) != 0) {
      if (b.epoch_graph) (void)hipGraphExecDestroy(b.epoch_graph);
      b.epoch_graph = nullptr;
      hipGraph_t g = nullptr;
      HIP_OR(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      int grid_used = 0;
      for (uint32_t i = 0; i < EPOCHS_PER_GRAPH && e == hipSuccess; ++i) {
        e = launch_compact(c->stream, b.d_out, b.n_txns, a.max_attempts, b.d_list, c->d_ctl);
        if (e == hipSuccess)
          e = launch_txn(c->stream, b.scheme, (int)lanes, (int)b.max_ops, (int)wpw, (int)p.grid, strict, latch, a,
                         c->n_cu, &grid_used);
      }
      const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
      if (e != hipSuccess) {
        if (e2 == hipSuccess && g) (void)hipGraphDestroy(g);
        return launch_error(c, e);
      }
      if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
      e = hipGraphInstantiate(&b.epoch_graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b.epoch_graph = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
      }
      std::memcpy(b.epoch_key, key, sizeof key);
      b.epoch_grid = grid_used;
    }
    first_grid = b.epoch_grid;
    uint64_t done_before = 0;
    for (;;) {
      HIP_OR(c, hipEventRecord(c->ev[1], c->stream));
      HIP_OR(c, hipGraphLaunch(b.epoch_graph, c->stream));
      HIP_OR(c, hipEventRecord(c->ev[2], c->stream));
      HIP_OR(c, hipStreamSynchronize(c->stream));
      float ms = 0;
      HIP_OR(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
      kernel_ms += ms;
      epochs += EPOCHS_PER_GRAPH;
      HIP_OR(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
      const uint64_t done = h.stats[DS_COMMITTED] + h.stats[DS_GAVE_UP];
      if (done >= b.n_txns || h.stop) break;
      if (epochs >= max_epochs) {
        epoch_limit = true;
        break;
      }
      // fewer than 1/256 of the pending transactions committed in four epochs:
      // the epochs are stalled on conflicts; finish with the plain passes
      const uint64_t pending = b.n_txns - done;
      if ((done - done_before) * 256 < pending || done == done_before) {
        // continue as a plain run would: same grid, then 8x smaller passes
        cc_status st = plain_passes(b.epoch_grid, wpw, false);
        if (st) return st;
        break;
      }
      done_before = done;
    }
  } else if (b.n_txns) {
    // OCC's hot-row engine: the transactions that write the batch's engine
    // rows run first, alone, in one workgroup; the rest then run as usual
    // (plain mode only: serving also passes here, and the engine knows no arrivals)
    // By default only where its one workgroup pays: the most written row
    // written by at least a tenth of the transactions, transactions of at
    // most 32 ops, and no row left out nearly as hot.  Measured: Zipf 0.9
    // and 0.99 gain 1.7-1.8x; Zipf 0.6 (0.5% of the transactions write the
    // hottest row) and order-entry (8 warehouses: 6%; 1 warehouse: transactions
    // of up to 66 ops) lose 7-56%.
    const bool eng_default = hot_share >= 0.1 && b.max_ops <= 32 && b.eng_gain;
    const bool use_eng = b.scheme == CC_OCC && p.mode == CC_MODE_PLAIN && !latch && eng_fits && b.n_eng_txns &&
                         b.d_part && b.d_eng_desc &&
                         ((p.flags & CC_RUN_HOT_ENGINE) || (!(p.flags & CC_RUN_NO_HOT_ENGINE) && eng_default));
    if (use_eng) {
      EngineArgs e = b.eng;
      e.desc = b.d_eng_desc;
      e.n_txns = b.n_eng_txns;
      a.defer_after = 0;
      HIP_OR(c, hipEventRecord(c->ev[1], c->stream));
      int threads = 0;
      // one workgroup: as many wavefronts as the variant allows, unless the caller chose
      const hipError_t er =
          launch_engine_occ(c->stream, (int)eng_lanes, (int)b.max_ops, (int)p.waves_per_wg, strict, a, e, &threads);
      if (er != hipSuccess) return launch_error(c, er);
      HIP_OR(c, hipEventRecord(c->ev[2], c->stream));
      HIP_OR(c, hipStreamSynchronize(c->stream));
      float ms = 0;
      HIP_OR(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
      kernel_ms += ms;
      engine_ms = ms;
      engine_txns = b.n_eng_txns;
      ++passes;
      a.list = b.d_part + b.n_eng_txns;
      a.n_txns = b.n_txns - b.n_eng_txns;
    }
    if (a.n_txns) {
      cc_status st = plain_passes((int)p.grid, wpw, true);
      if (st) return st;
    }
  }
  HIP_OR(c, hipEventRecord(c->ev[3], c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  HIP_OR(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  float ms_run = 0;
  HIP_OR(c, hipEventElapsedTime(&ms_run, c->ev[0], c->ev[3]));
  std::memset(b.stats, 0, sizeof(b.stats));
  b.stats[CC_STAT_COMMITTED] = h.stats[DS_COMMITTED];
  b.stats[CC_STAT_ATTEMPTS] = h.stats[DS_ATTEMPTS];
  b.stats[CC_STAT_ABORT_LOCK] = h.stats[DS_ABORT_LOCK];
  b.stats[CC_STAT_ABORT_VALID] = h.stats[DS_ABORT_VALID];
  b.stats[CC_STAT_KERNEL_NS] = (uint64_t)(kernel_ms * 1e6);
  b.stats[CC_STAT_RUN_NS] = (uint64_t)((double)ms_run * 1e6);
  b.stats[CC_STAT_TICKETS] = h.ticket - p.ts_start;
  b.stats[CC_STAT_MAX_ATTEMPTS] = h.stats[DS_MAX_ATTEMPTS];
  b.stats[CC_STAT_PASSES] = passes;
  b.stats[CC_STAT_DEFERRED] = h.stats[DS_DEFERRED];
  b.stats[CC_STAT_ENGINE_TXNS] = engine_txns;
  b.stats[CC_STAT_ENGINE_ROWS] = engine_txns ? b.eng.n_rows : 0;
  b.stats[CC_STAT_ENGINE_NS] = (uint64_t)(engine_ms * 1e6);
  b.stats[CC_STAT_ENGINE_WAITS] = h.stats[DS_ENGINE_WAITS];
  b.stats[CC_STAT_GRID] = (uint64_t)first_grid;
  b.stats[CC_STAT_EPOCHS] = epochs;
  const double ns_per_tick = 1e6 / (double)c->wallclock_khz;
  b.stats[CC_STAT_T_USEFUL_NS] = (uint64_t)((double)h.stats[DS_T_USEFUL] * ns_per_tick);
  b.stats[CC_STAT_T_ABORT_NS] = (uint64_t)((double)h.stats[DS_T_ABORT] * ns_per_tick);
  b.stats[CC_STAT_T_WAIT_NS] = (uint64_t)((double)h.stats[DS_T_WAIT] * ns_per_tick);
  b.stats[CC_STAT_GAVE_UP] = h.stats[DS_GAVE_UP];
  b.stats[CC_STAT_ADMIT_WAITS] = h.stats[DS_ADMIT_WAITS];
  b.stats[CC_STAT_WD_WAITS] = h.stats[DS_WD_WAITS];
  b.stats[CC_STAT_HOT_ACQ] = h.stats[DS_HOT_ACQ];
  b.stats[CC_STAT_HOT_FAILED] = h.stats[DS_HOT_FAILED];
  b.stats[CC_STAT_HOT_HOLD_NS] = (uint64_t)((double)h.stats[DS_HOT_HOLD] * ns_per_tick);
  b.stats[CC_STAT_HOT_WRITES] = b.hot_writes;
  b.stats[CC_STAT_BLOCKED_WAITS] = h.stats[DS_BLOCKED_WAITS];
  b.stats[CC_STAT_VERSION_SLOTS] = b.node_slots;
  b.stats[CC_STAT_VERSION_MISSES] = h.stats[DS_VERSION_MISS];
  for (int i = 0; i < 4; ++i)
    b.stats[CC_STAT_OCC_R1_NS + i] = (uint64_t)((double)h.stats[DS_R1 + i] * ns_per_tick);
  b.stats[CC_STAT_INDEX_NS] = (uint64_t)((double)ms_index * 1e6);
  b.ran = true;
  if (b.n_txns && host_stats) {
    std::vector<cc_outcome> o(b.n_txns);
    HIP_OR(c, hipMemcpy(o.data(), b.d_out, b.n_txns * sizeof(cc_outcome), hipMemcpyDeviceToHost));
    if (p.mode == CC_MODE_SERVE)
      for (uint64_t t = 0; t < b.n_txns; ++t) o[t].commit_ns -= b.arrival_ns[t];
    latency_percentiles(o, &b.stats[CC_STAT_LAT_P50_NS], &b.stats[CC_STAT_LAT_P99_NS]);
  }
  if (h.stats[DS_LATCH_STUCK] || h.stop)
    return fail(c, CC_E_LIVELOCK, "a row latch was not obtained within the spin limit; table contents are undefined");
  if (h.stats[DS_TS_OVERFLOW]) return fail(c, CC_E_TS_OVERFLOW, "timestamp overflow during the run");
  if (epoch_limit) return fail(c, CC_E_LIVELOCK, "max_epochs reached with transactions pending");
  if (h.stats[DS_COMMITTED] != b.n_txns) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "%llu of %llu transactions committed (attempt limit reached)",
                  (unsigned long long)h.stats[DS_COMMITTED], (unsigned long long)b.n_txns);
    return fail(c, CC_E_LIVELOCK, msg);
  }
  return CC_OK;
}

extern "C" {

cc_status cc_run(cc_ctx *c, uint64_t batch_id, const cc_run_params *pp) {
  if (!c) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  Batch &b = it->second;
  cc_run_params p{};
  if (pp) p = *pp;
  const cc_status pst = check_run_params(c, b.scheme, p);
  if (pst) return pst;
  return run_batch(c, b, p, true);
}

cc_status cc_run_static(cc_ctx *c, const cc_txn *txns, uint64_t n_txns, const cc_op *ops, uint64_t n_ops, int scheme,
                        const cc_run_params *pp, cc_outcome *per_txn, int64_t *per_op_read, uint64_t *counters,
                        uint32_t n_counters) {
  if (!c) return CC_E_INVAL;
  if ((n_txns && (!txns || !per_txn)) || (n_ops && (!ops || !per_op_read)) || (n_counters && !counters))
    return fail(c, CC_E_INVAL, "null array");
  if (scheme != CC_OCC && scheme != CC_2PL_NW && scheme != CC_2PL_WD && scheme != CC_TO && scheme != CC_TICTOC)
    return fail(c, CC_E_INVAL, "cc_run_static runs CC_OCC, CC_2PL_NW, CC_2PL_WD, CC_TO and CC_TICTOC");
  cc_run_params p{};
  if (pp) p = *pp;
  const cc_status pst = check_run_params(c, scheme, p);
  if (pst) return pst;
  if (p.mode != CC_MODE_PLAIN) return fail(c, CC_E_INVAL, "cc_run_static runs in CC_MODE_PLAIN only");
  if (p.flags & CC_RUN_LATCH) return fail(c, CC_E_INVAL, "cc_run_static does not take CC_RUN_LATCH");
  if (n_txns > CC_STATIC_MAX_TXNS || n_ops > CC_STATIC_MAX_OPS)
    return fail(c, CC_E_RANGE, "batch larger than the static scratch (CC_STATIC_MAX_TXNS, CC_STATIC_MAX_OPS)");
  if (!c->frozen) return fail(c, CC_E_STATE, "load the tables before running a batch");
  if (!c->d_static) return fail(c, CC_E_STATE, "no static scratch on this context's device");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  if (!device_range(c, txns, n_txns * sizeof(cc_txn)) || !device_range(c, ops, n_ops * sizeof(cc_op)) ||
      !device_range(c, per_txn, n_txns * sizeof(cc_outcome)) || !device_range(c, per_op_read, n_ops * sizeof(int64_t)))
    return fail(c, CC_E_INVAL, "arrays must lie in device memory of the context's device");
  unsigned char *sc = c->d_static;
  Batch b;
  b.scheme = scheme;
  b.n_txns = n_txns;
  b.n_ops = n_ops;
  b.d_ops = (DevOp *)(sc + STATIC_OFF_OPS);
  b.d_txns = (DevTxn *)(sc + STATIC_OFF_TXNS);
  b.d_list = (uint32_t *)(sc + STATIC_OFF_LIST);
  b.d_out = (DevOutcome *)per_txn;
  b.d_reads = per_op_read;
  IngestArgs ia{};
  ia.txns = txns;
  ia.ops = ops;
  ia.op_keys = nullptr;
  ia.n_txns = n_txns;
  ia.n_ops = n_ops;
  ia.n_tables = (uint32_t)c->tables.size();
  for (uint32_t t = 0; t < ia.n_tables; ++t) {
    const Table &tb = c->tables[t];
    ia.tab[t] = IngestTable{tb.n_rows, tb.row_base, tb.elem_base, tb.n_fields, 0u};
  }
  ia.dops = b.d_ops;
  ia.dtx = b.d_txns;
  ia.owner = (uint32_t *)(sc + STATIC_OFF_OWNER);
  ia.meta = nullptr;
  ia.rows0 = nullptr;
  ia.out = (uint64_t *)(sc + STATIC_OFF_INGEST);
  uint64_t res[INGEST_N] = {};
  hipError_t e = launch_ingest(c->stream, ia);
  if (e == hipSuccess) e = launch_fill_zero(c->stream, per_op_read, n_ops);
  if (e == hipSuccess) e = hipMemcpyAsync(res, ia.out, sizeof res, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch ingest");
  if (res[INGEST_ERR] != ~0ull) {
    const uint64_t w = res[INGEST_ERR];
    const cc_status code = -(cc_status)(w & 15u);
    return fail(c, code, std::string(ingest_message((uint32_t)((w >> 4) & 0xFFFu))) + " (transaction " +
                             std::to_string(w >> 16) + ")");
  }
  b.max_ops = (uint32_t)res[INGEST_MAX_OPS];
  b.has_slot = res[INGEST_HAS_SLOT] != 0;
  const cc_status st = run_batch(c, b, p, false);
  for (uint32_t i = 0; i < n_counters; ++i) counters[i] = i < CC_N_STATS ? b.stats[i] : 0;
  return st;
}

cc_status cc_fetch_outcomes(cc_ctx *c, uint64_t batch_id, cc_outcome *per_txn, int64_t *per_op, int on_device) {
  if (!c) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  Batch &b = it->second;
  if (!b.ran) return fail(c, CC_E_STATE, "batch has not been run");
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (per_txn && b.n_txns) HIP_OR(c, hipMemcpyAsync(per_txn, b.d_out, b.n_txns * sizeof(cc_outcome), k, c->stream));
  if (per_op && b.n_ops) HIP_OR(c, hipMemcpyAsync(per_op, b.d_reads, b.n_ops * sizeof(int64_t), k, c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  return CC_OK;
}

cc_status cc_set_arrivals(cc_ctx *c, uint64_t batch_id, const int64_t *arrival_ns, uint64_t n) {
  if (!c || (n && !arrival_ns)) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  Batch &b = it->second;
  if (n != b.n_txns) return fail(c, CC_E_INVAL, "one arrival time per transaction");
  std::vector<int64_t> ticks(std::max<uint64_t>(n, 1), 0);
  for (uint64_t t = 0; t < n; ++t) {
    if (arrival_ns[t] < 0 || (t && arrival_ns[t] < arrival_ns[t - 1]))
      return fail(c, CC_E_INVAL, "arrival times must be non-negative and non-decreasing");
    ticks[t] = (int64_t)((double)arrival_ns[t] * (double)c->wallclock_khz / 1e6);
  }
  if (!activate(c)) return fail(c, CC_E_HIP, "hipSetDevice failed");
  if (!b.d_arrival) HIP_OR(c, hipMalloc(&b.d_arrival, ticks.size() * sizeof(int64_t)));
  HIP_OR(c, hipMemcpyAsync(b.d_arrival, ticks.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIP_OR(c, hipStreamSynchronize(c->stream));
  b.arrival_ns.assign(arrival_ns, arrival_ns + n);
  return CC_OK;
}

cc_status cc_stats(cc_ctx *c, uint64_t batch_id, uint64_t *counters, uint32_t n) {
  if (!c || (!counters && n)) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  for (uint32_t i = 0; i < n && i < CC_N_STATS; ++i) counters[i] = it->second.stats[i];
  return CC_OK;
}

cc_status cc_release_batch(cc_ctx *c, uint64_t batch_id) {
  if (!c) return CC_E_INVAL;
  auto it = c->batches.find(batch_id);
  if (it == c->batches.end()) return fail(c, CC_E_NOBATCH, "unknown batch");
  activate(c);
  (void)hipStreamSynchronize(c->stream);
  free_batch(it->second);
  c->batches.erase(it);
  return CC_OK;
}

}  // extern "C"
