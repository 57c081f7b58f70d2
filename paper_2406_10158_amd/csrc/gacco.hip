// Conflict-graph ordering (GaccO): a deterministic scheme.  The paper's
// description (Section 2, "Conflict Graph Ordering"; Section 3, "Conflict
// Graph Ordering"): preprocessing gathers the (transaction, data item) pairs
// of the batch into an access table, orders every item's accesses by
// transaction id and builds a lock table that records which transaction
// currently owns each item; during execution an access waits until the item
// comes to its transaction, reads and writes alike, and passes the item on
// when it is done.  The serial order is therefore the transaction-id order
// and nothing ever aborts.
//
// gfx950 design.
//  * Access table: one 32-bit key per operation (its global row, or a
//    sentinel for operations that are not the first of their row group in
//    the transaction), the operation index as value.  The batch's operations
//    are stored in transaction order, so a stable sort by row leaves every
//    row's accesses in transaction order.
//  * Sort: least-significant-digit radix sort, 8-bit digits, as many passes
//    as the row ids need (3 for up to 16.7M rows).  Per pass: a tile
//    histogram kernel, an exclusive scan of the digit-major histogram table,
//    and a scatter kernel that ranks keys stably inside a 4,096-key tile with
//    wavefront ballots (8 ballots match the lanes holding the same digit) and
//    per-wavefront digit counters in LDS.  The paper uses a library sort and
//    prefix sum here; these are written for 64-lane wavefronts instead.
//  * Lock table: the row's control word holds a turn counter, initialised to
//    the position of the row's first access in the sorted table; the access
//    at sorted position p runs when the word equals p and releases by storing
//    p + 1.  Each row-group leader gets its position (rank) by a scatter.
//  * Execution: persistent teams of L lanes take transactions in id order
//    from a device counter, so every transaction a team waits for has
//    already been taken by a running wavefront and the oldest unfinished
//    transaction can always proceed.  A team polls the words of its waiting
//    rows, runs each row group as soon as its row comes to it, and releases
//    the row at once (not at the end of the transaction): a hot row is held
//    only for the load, the store and one ordering point.  Between polls a
//    waiting team sleeps in proportion to the number of accesses still
//    queued ahead of it on the row, so that the teams queued on a hot row do
//    not flood its word with loads.
#include "device.h"

namespace cce {

// ---------------------------------------------------------------------------
// access table
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gacco_keys_kernel(const DevOp *ops, uint64_t n_ops, uint32_t sentinel,
                                                         uint32_t *keys, uint32_t *vals) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ops) return;
  const uint32_t rk = ops[i].rowk;
  keys[i] = (rk & FOLLOWER_BIT) ? sentinel : (rk & ROW_MASK);
  vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// radix sort (stable, LSD, 8-bit digits) of (key, value) pairs
// ---------------------------------------------------------------------------
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_PER_LANE = 16;
constexpr int RS_TILE = RS_THREADS * RS_PER_LANE;  // keys per tile
constexpr int RS_RADIX = 256;
static_assert(RS_THREADS == RS_RADIX, "one thread per digit in the tile scans");

// Digit histogram of each tile, stored digit-major: hist[d * n_tiles + tile].
__global__ void __launch_bounds__(RS_THREADS) rs_hist_kernel(const uint32_t *keys, uint64_t n, int shift,
                                                             uint32_t *hist, uint32_t n_tiles) {
  __shared__ uint32_t cnt[RS_RADIX];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
  for (int j = 0; j < RS_PER_LANE; ++j) {
    const uint64_t i = base + (uint64_t)j * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (RS_RADIX - 1)], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of a workgroup's values (one per thread, RS_THREADS threads);
// returns the thread's exclusive prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds_waves, uint32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) lds_waves[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    const uint32_t s = lds_waves[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();  // lds_waves may be reused by the caller
  *total = all;
  return before + inc - v;
}

constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_CHUNK = RS_THREADS * SCAN_PER_THREAD;

// Pass 1 of the scan: the sum of each chunk.
__global__ void __launch_bounds__(RS_THREADS) scan_sum_kernel(const uint32_t *in, uint64_t m, uint32_t *partial) {
  __shared__ uint32_t lw[RS_WAVES];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t s = 0;
  for (int j = 0; j < SCAN_PER_THREAD; ++j)
    if (base + j < m) s += in[base + j];
  uint32_t total = 0;
  (void)block_exclusive_scan(s, lw, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Pass 2: exclusive scan of the chunk sums in one workgroup.
__global__ void __launch_bounds__(RS_THREADS) scan_partials_kernel(uint32_t *partial, uint32_t n_chunks) {
  __shared__ uint32_t lw[RS_WAVES];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < n_chunks; base += RS_THREADS) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < n_chunks ? partial[i] : 0u;
    uint32_t total = 0;
    const uint32_t ex = block_exclusive_scan(v, lw, &total);
    if (i < n_chunks) partial[i] = carry + ex;
    carry += total;
  }
}

// Pass 3: exclusive scan inside each chunk, offset by the chunk's prefix.
__global__ void __launch_bounds__(RS_THREADS) scan_apply_kernel(uint32_t *data, uint64_t m, const uint32_t *partial) {
  __shared__ uint32_t lw[RS_WAVES];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    v[j] = base + j < m ? data[base + j] : 0u;
    s += v[j];
  }
  uint32_t total = 0;
  uint32_t run = partial[blockIdx.x] + block_exclusive_scan(s, lw, &total);
#pragma unroll
  for (int j = 0; j < SCAN_PER_THREAD; ++j) {
    if (base + j < m) data[base + j] = run;
    run += v[j];
  }
}

// Stable scatter of one tile: wavefront w ranks keys [w*1024, (w+1)*1024) of
// the tile in 16 chunks of 64, in order, keeping per-wavefront digit counts
// in LDS; the tile's digit offsets then place wavefront w after w-1.
__global__ void __launch_bounds__(RS_THREADS) rs_scatter_kernel(const uint32_t *kin, const uint32_t *vin,
                                                                uint32_t *kout, uint32_t *vout, uint64_t n,
                                                                int shift, const uint32_t *hist,
                                                                uint32_t n_tiles) {
  __shared__ uint32_t cnt[RS_WAVES][RS_RADIX];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < RS_WAVES * RS_RADIX; i += RS_THREADS) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)w * (RS_TILE / RS_WAVES);
  const uint64_t below_me = (1ull << lane) - 1ull;
  uint32_t key[RS_PER_LANE], val[RS_PER_LANE], pos[RS_PER_LANE];
#pragma unroll
  for (int j = 0; j < RS_PER_LANE; ++j) {
    const uint64_t i = base + (uint64_t)j * 64 + lane;
    key[j] = i < n ? kin[i] : 0u;
    val[j] = i < n ? vin[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < RS_PER_LANE; ++j) {
    const bool ok = base + (uint64_t)j * 64 + lane < n;
    const uint32_t d = (key[j] >> shift) & (RS_RADIX - 1);
    uint64_t same = ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = ballot(bit);
      same &= bit ? bb : ~bb;
    }
    const uint32_t earlier = (uint32_t)__popcll(same & below_me);
    uint32_t c = 0;
    if (ok) c = cnt[w][d];
    pos[j] = c + earlier;
    // the first lane of each digit group advances the count after every lane
    // of the group has read it (one wavefront, LDS operations in order)
    if (ok && earlier == 0) cnt[w][d] = c + (uint32_t)__popcll(same);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = hist[(uint64_t)d * n_tiles + blockIdx.x];
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww) {
      const uint32_t c = cnt[ww][d];
      cnt[ww][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_PER_LANE; ++j) {
    if (base + (uint64_t)j * 64 + lane < n) {
      const uint32_t d = (key[j] >> shift) & (RS_RADIX - 1);
      const uint32_t dst = cnt[w][d] + pos[j];
      if (dst < n) {  // always true for a consistent histogram; never write outside the buffers
        kout[dst] = key[j];
        vout[dst] = val[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// lock table: turn counters and per-access ranks
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gacco_lock_table_kernel(const uint32_t *keys, const uint32_t *vals, uint64_t n,
                                                               uint32_t sentinel, uint64_t *words, uint32_t *rank) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i], v = vals[i];
  if (k >= sentinel || v >= n) return;  // followers (and nothing else) carry the sentinel
  if (i == 0 || keys[i - 1] != k) words[k] = i;  // the row's first access owns it
  rank[v] = (uint32_t)i;
}


// Shared reads (CC_RUN_SHARED_READS): each row's word holds two counters,
// accesses done (high 32 bits) and writes done (low 32 bits).  A write waits
// until every earlier access of its row is done, a read only until every
// earlier write is; the reads between two writes run together.
// First pass: write flags of the sorted accesses, and each row's start.
__global__ void __launch_bounds__(256) gacco_shared_flags_kernel(const uint32_t *keys, const uint32_t *vals,
                                                                 uint64_t n, uint32_t sentinel, const DevOp *ops,
                                                                 uint64_t *words, uint32_t *wflag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i], v = vals[i];
  const bool real = k < sentinel && v < n;
  wflag[i] = (real && op_written(ops[v].rowk)) ? 1u : 0u;
  if (real && (i == 0 || keys[i - 1] != k)) words[k] = i;  // the row's first position, for the next pass
}

// Second pass (after an exclusive scan turned the flags into "writes before
// position i"): each leader's threshold -- accesses before it in its row for
// a write, writes before it in its row for a read.
__global__ void __launch_bounds__(256) gacco_shared_rank_kernel(const uint32_t *keys, const uint32_t *vals,
                                                                uint64_t n, uint32_t sentinel, const DevOp *ops,
                                                                const uint64_t *words, const uint32_t *wbefore,
                                                                uint32_t *rank) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i], v = vals[i];
  if (k >= sentinel || v >= n) return;
  const uint64_t start = words[k];
  if (start > i) return;  // not reachable for a consistent table
  rank[v] = op_written(ops[v].rowk) ? (uint32_t)(i - start) : wbefore[i] - wbefore[start];
}

// Per-row positions (PREP_LOCAL, GPUTx's packed rank state): after the lock
// table has put each row's first position in its word, every leader's place
// in its row's list becomes its position minus that start.
__global__ void __launch_bounds__(256) gacco_local_rank_kernel(const uint32_t *keys, const uint32_t *vals, uint64_t n,
                                                               uint32_t sentinel, const uint64_t *words,
                                                               uint32_t *rank) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i], v = vals[i];
  if (k >= sentinel || v >= n) return;
  const uint64_t start = words[k];
  if (start > i) return;  // not reachable for a consistent table
  rank[v] = (uint32_t)(i - start);
}

// Third pass: both counters of every accessed row start at zero.
__global__ void __launch_bounds__(256) gacco_shared_clear_kernel(const uint32_t *keys, uint64_t n, uint32_t sentinel,
                                                                 uint64_t *words) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (k < sentinel && (i == 0 || keys[i - 1] != k)) words[k] = 0;
}

// Exclusive scan of m 32-bit values in place (partial: (m + 4095) / 4096 + 1 words).
static void exclusive_scan_u32(hipStream_t s, uint32_t *data, uint64_t m, uint32_t *partial) {
  const uint64_t chunks = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
  hipLaunchKernelGGL(scan_sum_kernel, dim3((unsigned)chunks), dim3(RS_THREADS), 0, s, data, m, partial);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(RS_THREADS), 0, s, partial, (uint32_t)chunks);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)chunks), dim3(RS_THREADS), 0, s, data, m, partial);
}

__global__ void __launch_bounds__(64) gacco_reset_kernel(Ctl *ctl) {
  if (threadIdx.x == 0) ctl->stop = 0;
}

uint64_t radix_sort_scratch_words(uint64_t n);
uint64_t gacco_scratch_words(uint64_t n_ops) { return 2 * n_ops + radix_sort_scratch_words(n_ops); }

hipError_t radix_sort_pairs(hipStream_t s, uint32_t *keys, uint32_t *vals, uint64_t n, int bits, uint32_t *scratch,
                            uint32_t **keys_out, uint32_t **vals_out) {
  const uint64_t tiles = (n + RS_TILE - 1) / RS_TILE;
  const uint64_t m = tiles * RS_RADIX;
  const uint64_t chunks = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
  if (tiles > 0xFFFFFFFFull || chunks > 0xFFFFFFFFull) return hipErrorInvalidValue;
  uint32_t *ka = keys, *va = vals, *kb = scratch, *vb = kb + n, *hist = vb + n, *partial = hist + m;
  for (int shift = 0; shift < bits && n; shift += 8) {
    hipLaunchKernelGGL(rs_hist_kernel, dim3((unsigned)tiles), dim3(RS_THREADS), 0, s, ka, n, shift, hist,
                       (uint32_t)tiles);
    hipLaunchKernelGGL(scan_sum_kernel, dim3((unsigned)chunks), dim3(RS_THREADS), 0, s, hist, m, partial);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(RS_THREADS), 0, s, partial, (uint32_t)chunks);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)chunks), dim3(RS_THREADS), 0, s, hist, m, partial);
    hipLaunchKernelGGL(rs_scatter_kernel, dim3((unsigned)tiles), dim3(RS_THREADS), 0, s, ka, va, kb, vb, n, shift,
                       hist, (uint32_t)tiles);
    uint32_t *t = ka; ka = kb; kb = t;
    t = va; va = vb; vb = t;
  }
  *keys_out = ka;
  *vals_out = va;
  return hipGetLastError();
}

uint64_t radix_sort_scratch_words(uint64_t n) {
  const uint64_t tiles = (n + RS_TILE - 1) / RS_TILE;
  const uint64_t m = tiles * RS_RADIX;
  const uint64_t chunks = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
  return 2 * n + m + chunks + 1;
}

hipError_t gacco_prepare(hipStream_t s, const DevOp *ops, uint64_t n_ops, uint32_t sentinel, uint64_t *words,
                         uint32_t *rank, uint32_t *scratch, Ctl *ctl, int mode) {
  hipLaunchKernelGGL(gacco_reset_kernel, dim3(1), dim3(64), 0, s, ctl);
  if (n_ops == 0) return hipGetLastError();
  // scratch: [ka | va | radix scratch: kb | vb | histogram | partial sums]
  uint32_t *ka = scratch, *va = ka + n_ops, *rs = va + n_ops, *sorted_k = nullptr, *sorted_v = nullptr;
  const unsigned blocks = (unsigned)((n_ops + 255) / 256);
  hipLaunchKernelGGL(gacco_keys_kernel, dim3(blocks), dim3(256), 0, s, ops, n_ops, sentinel, ka, va);
  int bits = 0;
  while (bits < 32 && (sentinel >> bits) != 0) ++bits;
  hipError_t e = radix_sort_pairs(s, ka, va, n_ops, bits, rs, &sorted_k, &sorted_v);
  if (e != hipSuccess) return e;
  if (mode != PREP_SHARED) {
    hipLaunchKernelGGL(gacco_lock_table_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, sorted_v, n_ops, sentinel,
                       words, rank);
    if (mode == PREP_LOCAL) {
      // places within each row, and every accessed row's word starts at zero
      hipLaunchKernelGGL(gacco_local_rank_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, sorted_v, n_ops, sentinel,
                         words, rank);
      hipLaunchKernelGGL(gacco_shared_clear_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, n_ops, sentinel, words);
    }
    return hipGetLastError();
  }
  // the key/value pair the sort did not end in is free, and so is the histogram
  uint32_t *wflag = sorted_k == ka ? rs : ka;
  uint32_t *partial = rs + 2 * n_ops;
  hipLaunchKernelGGL(gacco_shared_flags_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, sorted_v, n_ops, sentinel,
                     ops, words, wflag);
  exclusive_scan_u32(s, wflag, n_ops, partial);
  hipLaunchKernelGGL(gacco_shared_rank_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, sorted_v, n_ops, sentinel,
                     ops, words, wflag, rank);
  hipLaunchKernelGGL(gacco_shared_clear_kernel, dim3(blocks), dim3(256), 0, s, sorted_k, n_ops, sentinel, words);
  return hipGetLastError();
}

}  // namespace cce
