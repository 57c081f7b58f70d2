// Memory micro-benchmarks that bound the transaction kernels: the engine's
// hot path is random 8-byte accesses and 64-bit device atomics, so its
// roofline is set by how many of those the memory system sustains, not by
// streaming bandwidth or arithmetic.  Each probe times one kernel with HIP
// events; addresses come from a hash of the op index (no index traffic).
#include <algorithm>

#include "engine.h"

namespace cce {

__device__ __forceinline__ uint64_t hash64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// 16-byte streaming copy src -> dst.
__global__ void __launch_bounds__(256) probe_stream(const uint4 *src, uint4 *dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Random 8-byte accesses over `words` words (any count: the word index is the
// high half of hash x words, uniform over [0, words)), or, with `idx`, at the
// caller's word indices idx[i] for op i (threads take ops i, i + threads, ...).
// mode 0: agent-scope loads   1: plain loads   2: agent-scope stores
//      3: agent-scope fetch_or   4: agent-scope fetch_add on one word (every lane)
//      5: agent-scope fetch_add on one word, one per wavefront
template <int MODE>
__global__ void __launch_bounds__(256) probe_random(uint64_t *words, uint64_t n_words, uint64_t per_thread,
                                                   const uint64_t *idx, uint64_t n_idx, uint64_t *sink) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t threads = (uint64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (uint64_t j = 0; j < per_thread; j += 4) {
    uint64_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint64_t w;
      bool on = true;
      if (idx) {
        const uint64_t i = (j + u) * threads + tid;
        on = i < n_idx;
        w = on ? idx[i] : 0;
      } else {
        w = __umul64hi(hash64((tid << 24) ^ (j + u)), n_words);
      }
      v[u] = 0;
      if (!on) continue;
      if constexpr (MODE == 0) {
        v[u] = __hip_atomic_load(words + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if constexpr (MODE == 1) {
        v[u] = words[w];
      } else if constexpr (MODE == 2) {
        __hip_atomic_store(words + w, j + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if constexpr (MODE == 3) {
        v[u] = __hip_atomic_fetch_or(words + w, 1ull << (u + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if constexpr (MODE == 4) {
        v[u] = __hip_atomic_fetch_add(words, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (__lane_id() == 0) v[u] = __hip_atomic_fetch_add(words, 64ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    acc += v[0] ^ v[1] ^ v[2] ^ v[3];
  }
  if (acc == 0x5A5A5A5A5A5A5A5Aull) sink[tid & 1023] = acc;  // keeps the loads live
}

// The two sides of a hand-off probe: lane 0 of block 0 and lane 0 of block
// `peer`.  Blocks are dealt round-robin to the 8 XCDs, so peer 1 is on another
// XCD and peer 8 on the same XCD (another CU); peer 0 puts the two sides in
// the first two wavefronts of block 0, which share one CU.  -1: not a side.
__device__ __forceinline__ int handoff_side(int peer) {
  if (threadIdx.x % 64 != 0) return -1;
  const int wave = (int)threadIdx.x / 64;
  if (peer == 0) return blockIdx.x == 0 && wave < 2 ? wave : -1;
  if (wave != 0) return -1;
  if (blockIdx.x == 0) return 0;
  if ((int)blockIdx.x == peer) return 1;
  return -1;
}

// Ping-pong on one word between the two sides (handoff_side).  Each side
// waits for its turn with agent-scope loads, bounded by `spin_limit` polls per
// turn; on exhaustion it records an error and stops, and so does the other
// side once its own bounded wait runs out.
__global__ void __launch_bounds__(128) probe_handoff(uint64_t *flag, uint64_t rounds, int peer, uint64_t spin_limit,
                                                     uint64_t *err) {
  const int side = handoff_side(peer);
  if (side < 0) return;
  for (uint64_t r = 0; r < rounds; ++r) {
    const uint64_t want = 2 * r + (uint64_t)side;
    uint64_t spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
      if (++spins > spin_limit) {
        __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    __hip_atomic_store(flag, want + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The OCC commit critical section on one hot row, handed back and forth
// between the two sides (handoff_side): wait until the row's
// word carries the previous round's version (bounded), then lock it with
// fetch_or, read the row's value and draw a ticket, re-read a second word
// (the validation read), store the new value, wait for completion and
// publish the word.  The time per round is the shortest interval between two
// commits on one row that this lock / ticket / validate / install sequence
// allows: the hot-row hand-off time t_h.
__global__ void __launch_bounds__(128) probe_commit_handoff(uint64_t *buf, uint64_t rounds, int peer,
                                                            uint64_t spin_limit, uint64_t *err) {
  const int side = handoff_side(peer);
  if (side < 0) return;
  uint64_t *word = buf, *value = buf + 64, *ticket = buf + 128, *other = buf + 192 + 16 * side;
  const uint64_t LOCKBIT = 1ull << 63;
  for (uint64_t r = (uint64_t)side; r < rounds; r += 2) {
    uint64_t spins = 0;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != r) {
      if (++spins > spin_limit) {
        __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    const uint64_t old = __hip_atomic_fetch_or(word, LOCKBIT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t v = __hip_atomic_load(value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t o = __hip_atomic_load(other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(value, v + 1 + (o == 0x5A5Aull ? t + old : 0ull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_store(word, r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The hot-row engine's commit critical section on one engine row, handed
// back and forth between two wavefronts of one workgroup: wait for the turn
// (an LDS word, bounded), take the row's LDS lock, draw a ticket from an LDS
// counter, load a validation word from LDS (the engine validates its other
// rows in an LDS table), store the new value in LDS and release the lock.
// The time per round is the shortest interval between two commits on one
// engine row: the engine's t_h.
__global__ void __launch_bounds__(128) probe_engine_handoff(uint64_t *buf, uint64_t rounds, uint64_t spin_limit,
                                                            uint64_t *err) {
  __shared__ uint32_t lk;
  __shared__ uint64_t turn, ticket, bucket[2];
  __shared__ int64_t value;
  if (threadIdx.x == 0) {
    lk = 0;
    turn = 0;
    ticket = 0;
    value = 0;
    bucket[0] = bucket[1] = (uint64_t)buf[0];
  }
  __syncthreads();
  if (threadIdx.x % 64 != 0) return;
  const uint64_t side = threadIdx.x / 64;
  for (uint64_t r = side; r < rounds; r += 2) {
    uint64_t spins = 0;
    while (__hip_atomic_load(&turn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != r) {
      if (++spins > spin_limit) {
        __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    uint32_t expect = 0;
    const bool got = __hip_atomic_compare_exchange_strong(&lk, &expect, 1u << 31, __ATOMIC_RELAXED,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const uint64_t t = __hip_atomic_fetch_add(&ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const uint64_t o = __hip_atomic_load(&bucket[side], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    value = value + 1 + (o == 0x5A5Aull ? (int64_t)t + got : 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    (void)__hip_atomic_fetch_and(&lk, ~(1u << 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_store(&turn, r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

__global__ void fill_kernel(uint64_t *p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t run_probe(hipStream_t s, int kind, uint64_t footprint_bytes, uint64_t n_ops, int peer,
                     const uint64_t *host_idx, double *ms_out, uint64_t *err_out, int n_cu) {
  *err_out = 0;
  const uint64_t words = footprint_bytes / sizeof(uint64_t) / 4 * 4;  // the stream copy moves 4-word chunks
  uint64_t *buf = nullptr, *aux = nullptr, *idx = nullptr;
  hipError_t e = hipMalloc(&buf, words * sizeof(uint64_t));
  if (e != hipSuccess) return e;
  e = hipMalloc(&aux, 8192 * sizeof(uint64_t));
  if (e == hipSuccess && host_idx) e = hipMalloc(&idx, std::max<uint64_t>(n_ops, 1) * sizeof(uint64_t));
  if (e == hipSuccess && host_idx && n_ops)
    e = hipMemcpyAsync(idx, host_idx, n_ops * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    if (aux) (void)hipFree(aux);
    if (idx) (void)hipFree(idx);
    return e;
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, s, buf, words, 0ull);
  hipLaunchKernelGGL(fill_kernel, dim3(32), dim3(256), 0, s, aux, 8192ull, 0ull);
  const unsigned grid = (unsigned)(n_cu * 8), block = 256;
  const uint64_t threads = (uint64_t)grid * block;
  uint64_t per = (n_ops + threads - 1) / threads;
  per = (per + 3) & ~3ull;
  if (per == 0) per = 4;
  const uint64_t n_idx = host_idx ? n_ops : 0;
  (void)hipEventRecord(a, s);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(probe_stream, dim3(grid * 4), dim3(256), 0, s, (const uint4 *)buf,
                         (uint4 *)(buf + words / 2), (uint64_t)(words / 4));
      break;
    case 1: hipLaunchKernelGGL(probe_random<0>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 2: hipLaunchKernelGGL(probe_random<1>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 3: hipLaunchKernelGGL(probe_random<2>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 4: hipLaunchKernelGGL(probe_random<3>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 5: hipLaunchKernelGGL(probe_random<4>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 6: hipLaunchKernelGGL(probe_random<5>, dim3(grid), dim3(block), 0, s, buf, words, per, idx, n_idx, aux); break;
    case 7:
      hipLaunchKernelGGL(probe_handoff, dim3((unsigned)(peer + 1)), dim3(128), 0, s, buf, n_ops, peer,
                         (uint64_t)1 << 20, aux + 4096);
      break;
    case 8:
      hipLaunchKernelGGL(probe_commit_handoff, dim3((unsigned)(peer + 1)), dim3(128), 0, s, buf, n_ops, peer,
                         (uint64_t)1 << 20, aux + 4096);
      break;
    case 9:
      hipLaunchKernelGGL(probe_engine_handoff, dim3(1), dim3(128), 0, s, buf, n_ops, (uint64_t)1 << 20, aux + 4096);
      break;
    default:
      break;
  }
  e = hipGetLastError();
  (void)hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (e == hipSuccess && (kind == 7 || kind == 8 || kind == 9)) e = hipMemcpy(err_out, aux + 4096, sizeof(uint64_t), hipMemcpyDeviceToHost);
  *ms_out = ms;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(buf);
  (void)hipFree(aux);
  if (idx) (void)hipFree(idx);
  return e;
}

}  // namespace cce
