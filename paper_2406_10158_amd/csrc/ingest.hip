// Device-side batch ingest: validate a batch that is already in device memory
// (cc_submit_batch with on_device != 0) and pack it into the engine's
// operation and transaction descriptors, without a round trip through the
// host.  The rules and status codes are the host path's (api.cpp,
// validate_and_pack), in the same order, so that both report the same status
// for the same arrays: per transaction, the first failing check in program
// order; over the batch, the lowest-numbered malformed transaction.
//
// Three kernels, one thread per operation or transaction:
//   ingest_fill   default descriptors (an op no transaction names is a
//                 follower, so it never enters GaccO's access table) and the
//                 per-op owner slot set to "none";
//   ingest_claim  each transaction whose header is well formed records
//                 itself as an owner of its ops (atomic minimum), so that an
//                 op named by two transactions is reported at the later one,
//                 as the host's in-order scan does;
//   ingest_pack   checks every op, builds the row groups (leader / follower,
//                 written), rejects repeated rows and fields, writes the
//                 descriptors and reduces max ops, slot use and ordering.
#include "device.h"

namespace cce {

namespace {

// error word: (transaction << 16) | (message << 4) | code, minimum wins
__device__ __forceinline__ void report(IngestArgs &a, uint64_t t, uint32_t msg, uint32_t code) {
  atomicMin((unsigned long long *)&a.out[INGEST_ERR], (unsigned long long)((t << 16) | (msg << 4) | code));
}

__device__ __forceinline__ bool header_ok(const IngestArgs &a, const cc_txn &x, uint32_t *msg) {
  if (x.reserved != 0) { *msg = INGEST_MSG_RESERVED; return false; }
  if (x.n_ops > CC_MAX_OPS_PER_TXN) { *msg = INGEST_MSG_TOO_MANY; return false; }
  if (x.first_op > a.n_ops || x.n_ops > a.n_ops - x.first_op) { *msg = INGEST_MSG_OP_RANGE; return false; }
  return true;
}

}  // namespace

__global__ void __launch_bounds__(256) ingest_fill_kernel(IngestArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ops) return;
  DevOp d;
  d.rowk = FOLLOWER_BIT;
  d.elem = 0;
  d.arg = 0;
  a.dops[i] = d;
  a.owner[i] = 0xFFFFFFFFu;
  if (a.meta) {
    a.meta[i] = 0;
    a.rows0[i] = a.ops[i].row;
  }
}

__global__ void __launch_bounds__(256) ingest_claim_kernel(IngestArgs a) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_txns) return;
  const cc_txn x = a.txns[t];
  uint32_t msg = 0;
  if (!header_ok(a, x, &msg)) return;
  for (uint32_t i = 0; i < x.n_ops; ++i) atomicMin(&a.owner[x.first_op + i], (uint32_t)t);
}

__global__ void __launch_bounds__(256) ingest_pack_kernel(IngestArgs a) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_txns) return;
  const cc_txn x = a.txns[t];
  uint32_t msg = 0;
  if (!header_ok(a, x, &msg)) {
    report(a, t, msg, (uint32_t)-CC_E_INVAL);
    return;
  }
  if (t > 0 && x.first_op < a.txns[t - 1].first_op) atomicOr((unsigned long long *)&a.out[INGEST_UNORDERED], 1ull);
  for (uint32_t i = 0; i < x.n_ops; ++i) {
    if (a.owner[x.first_op + i] != (uint32_t)t) {
      report(a, t, INGEST_MSG_SHARED, (uint32_t)-CC_E_INVAL);
      return;
    }
  }
  // an op's row identity: its key on an indexed table (keyed batch), else its row
  auto keyed = [&](const cc_op &o) { return a.op_keys != nullptr && o.table < a.n_tables && a.tab[o.table].indexed; };
  auto ident = [&](uint64_t op, const cc_op &o) -> int64_t { return keyed(o) ? a.op_keys[op] : (int64_t)o.row; };
  uint32_t group_start = 0;
  bool group_written = false, slot = false, any_keyed = false;
  cc_op prev{};
  int64_t prev_id = 0;
  for (uint32_t i = 0; i < x.n_ops; ++i) {
    const uint64_t op = x.first_op + i;
    const cc_op o = a.ops[op];
    if (o.table >= a.n_tables) { report(a, t, INGEST_MSG_TABLE, (uint32_t)-CC_E_RANGE); return; }
    const IngestTable &tb = a.tab[o.table];
    const bool kd = keyed(o);
    if (kd && o.row != 0) { report(a, t, INGEST_MSG_KEYED_ROW, (uint32_t)-CC_E_INVAL); return; }
    if ((!kd && o.row >= tb.n_rows) || o.field >= tb.n_fields) {
      report(a, t, INGEST_MSG_ROW_FIELD, (uint32_t)-CC_E_RANGE);
      return;
    }
    if (o.kind > CC_WRITE_SLOT) { report(a, t, INGEST_MSG_KIND, (uint32_t)-CC_E_INVAL); return; }
    if (o.kind == CC_WRITE_SLOT) {
      slot = true;
      if ((uint32_t)(o.arg & 0xFF) >= i) { report(a, t, INGEST_MSG_SLOT_SRC, (uint32_t)-CC_E_INVAL); return; }
    }
    const int64_t id = ident(op, o);
    const bool follower = i > 0 && prev.table == o.table && prev_id == id;
    if (!follower) {
      if (group_written)
        for (uint32_t j = group_start; j < i; ++j) a.dops[x.first_op + j].rowk |= WRITTEN_BIT;
      group_start = i;
      group_written = false;
    } else {
      for (uint32_t j = group_start; j < i; ++j)
        if (a.ops[x.first_op + j].field == o.field) {
          report(a, t, INGEST_MSG_DUP_FIELD, (uint32_t)-CC_E_DUPROW);
          return;
        }
    }
    group_written |= o.kind != CC_READ;
    const uint64_t grow = kd ? 0 : tb.row_base + o.row;
    DevOp d;
    d.rowk = (uint32_t)grow | ((uint32_t)o.kind << KIND_SHIFT) | (follower ? FOLLOWER_BIT : 0u);
    d.elem = kd ? 0u : (uint32_t)(tb.elem_base + (uint64_t)o.row * tb.n_fields + o.field);
    d.arg = o.arg;
    a.dops[op] = d;
    if (kd) {
      a.meta[op] = META_KEYED | ((uint32_t)o.table << 16) | o.field;
      any_keyed = true;
    }
    prev = o;
    prev_id = id;
  }
  if (group_written)
    for (uint32_t j = group_start; j < x.n_ops; ++j) a.dops[x.first_op + j].rowk |= WRITTEN_BIT;
  // a (table, row) may start only one row group
  for (uint32_t i = 0; i < x.n_ops; ++i) {
    const uint64_t oi = x.first_op + i;
    if (a.dops[oi].rowk & FOLLOWER_BIT) continue;
    const cc_op p = a.ops[oi];
    const int64_t pid = ident(oi, p);
    for (uint32_t j = i + 1; j < x.n_ops; ++j) {
      const uint64_t oj = x.first_op + j;
      if (a.dops[oj].rowk & FOLLOWER_BIT) continue;
      const cc_op q = a.ops[oj];
      if (q.table == p.table && ident(oj, q) == pid) {
        report(a, t, INGEST_MSG_DUP_ROW, (uint32_t)-CC_E_DUPROW);
        return;
      }
    }
  }
  DevTxn dt;
  dt.first = (uint32_t)x.first_op;
  dt.n = x.n_ops;
  a.dtx[t] = dt;
  atomicMax((unsigned long long *)&a.out[INGEST_MAX_OPS], (unsigned long long)x.n_ops);
  if (slot) atomicOr((unsigned long long *)&a.out[INGEST_HAS_SLOT], 1ull);
  if (any_keyed) atomicOr((unsigned long long *)&a.out[INGEST_KEYED], 1ull);
}

__global__ void __launch_bounds__(64) ingest_reset_kernel(uint64_t *out) {
  if (threadIdx.x < INGEST_N) out[threadIdx.x] = threadIdx.x == INGEST_ERR ? ~0ull : 0ull;
}

hipError_t launch_ingest(hipStream_t s, const IngestArgs &a) {
  hipLaunchKernelGGL(ingest_reset_kernel, dim3(1), dim3(64), 0, s, a.out);
  const uint64_t bo = (a.n_ops + 255) / 256, bt = (a.n_txns + 255) / 256;
  if (bo) hipLaunchKernelGGL(ingest_fill_kernel, dim3((unsigned)bo), dim3(256), 0, s, a);
  if (bt) {
    hipLaunchKernelGGL(ingest_claim_kernel, dim3((unsigned)bt), dim3(256), 0, s, a);
    hipLaunchKernelGGL(ingest_pack_kernel, dim3((unsigned)bt), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace cce
