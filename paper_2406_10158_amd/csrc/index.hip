// Index lookups: keys to rows through a table's sorted-array index.
//
// The paper's index is a sorted array of the indexed column kept with the
// primary keys, searched by binary search (Section 3.4, "Index"); it also
// compares a B+ tree (Section 4.2, index experiment).  Here the keys of a
// keyed batch are resolved once per run, before the concurrency control
// starts and inside the measured window: read/write sets are fixed and keys
// never change (no inserts or deletes, Section 4.1), so resolving them in a
// separate pass gives the same rows as looking each one up inside the
// transaction, and the lookups of a batch run as one coalesced kernel.
//
//  * binary search: one lane per op, ~log2(n) dependent 8-byte loads;
//  * 16-way tree: one lane per op descends a static tree whose nodes are 16
//    consecutive keys (one 128-byte line, read as 8 16-byte loads): a 10M-key
//    index takes 7 dependent line loads instead of 24 dependent 8-byte loads,
//    and the upper levels stay in cache.  (A first version gave each op 16
//    lanes, one key each, and a ballot per level: 16x the wavefronts, and
//    slower than binary search, 3.5 ms against 2.2 ms for 16M lookups.)
#include "device.h"

namespace cce {

__device__ __forceinline__ void patch_op(DevOp *ops, uint64_t i, const IndexDesc &d, uint32_t row, uint32_t field) {
  DevOp o = ops[i];
  o.rowk = (o.rowk & ~ROW_MASK) | (uint32_t)(d.row_base + row);
  o.elem = (uint32_t)(d.elem_base + (uint64_t)row * d.n_fields + field);
  ops[i] = o;
}

__global__ void __launch_bounds__(256) index_bsearch_kernel(const int64_t *op_keys, const uint32_t *meta, DevOp *ops,
                                                           uint32_t *rows_out, uint64_t n_ops, const IndexDesc *idx,
                                                           Ctl *ctl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ops) return;
  const uint32_t m = meta[i];
  if (!(m & META_KEYED)) return;
  const IndexDesc &d = idx[(m >> 16) & 0xFF];
  const int64_t key = op_keys[i];
  uint64_t lo = 0, hi = d.n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (d.keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  const bool found = lo < d.n && d.keys[lo] == key;
  const uint32_t row = found ? d.rows[lo] : 0u;
  if (!found) atomicAdd((unsigned long long *)&ctl->stats[DS_INDEX_MISS], 1ull);
  rows_out[i] = row;
  patch_op(ops, i, d, row, m & 0xFF);
}

// The 16 entries of one tree node (one 128-byte line), as 8 16-byte loads.
__device__ __forceinline__ void load_node(const int64_t *p, int64_t (&e)[16]) {
#pragma unroll
  for (int j = 0; j < 16; j += 2) {
    const longlong2 v = *reinterpret_cast<const longlong2 *>(p + j);
    e[j] = v.x;
    e[j + 1] = v.y;
  }
}

__global__ void __launch_bounds__(256) index_tree_kernel(const int64_t *op_keys, const uint32_t *meta, DevOp *ops,
                                                        uint32_t *rows_out, uint64_t n_ops, const IndexDesc *idx,
                                                        Ctl *ctl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ops) return;
  const uint32_t m = meta[i];
  if (!(m & META_KEYED)) return;
  const IndexDesc &d = idx[(m >> 16) & 0xFF];
  const int64_t key = op_keys[i];
  bool miss = key == INT64_MAX;  // the padding value is not a key
  uint64_t node = 0;
  int64_t e[16];
  for (int l = (int)d.levels; l >= 1; --l) {
    load_node(d.tree + d.level_off[l] + node * 16, e);
    // the child is the first entry not below the key; none (every real
    // entry below it) means the key is above every key of the subtree.  A
    // miss continues from node 0, so that every load stays inside the levels.
    uint32_t below = 0, real = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      below += e[j] < key;
      real += e[j] != INT64_MAX;
    }
    if (below >= real) {
      miss = true;
      node = 0;
    } else {
      node = node * 16 + below;
    }
  }
  load_node(d.keys + node * 16, e);
  int hit = -1;
#pragma unroll
  for (int j = 15; j >= 0; --j)
    if (e[j] == key) hit = j;
  miss |= hit < 0;
  const uint32_t row = miss ? 0u : d.rows[node * 16 + (uint64_t)hit];
  if (miss) atomicAdd((unsigned long long *)&ctl->stats[DS_INDEX_MISS], 1ull);
  rows_out[i] = row;
  patch_op(ops, i, d, row, m & 0xFF);
}

hipError_t launch_index_lookup(hipStream_t s, bool tree, const int64_t *op_keys, const uint32_t *meta, DevOp *ops,
                               uint32_t *rows_out, uint64_t n_ops, const IndexDesc *idx, Ctl *ctl) {
  if (n_ops == 0) return hipSuccess;
  const uint64_t blocks = (n_ops + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  if (tree)
    hipLaunchKernelGGL(index_tree_kernel, dim3((unsigned)blocks), dim3(256), 0, s, op_keys, meta, ops, rows_out, n_ops,
                       idx, ctl);
  else
    hipLaunchKernelGGL(index_bsearch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, op_keys, meta, ops, rows_out,
                       n_ops, idx, ctl);
  return hipGetLastError();
}

}  // namespace cce
