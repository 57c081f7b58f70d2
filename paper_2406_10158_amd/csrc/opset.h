// Sets of a transaction's operation indices held in every lane of its team,
// built from wavefront ballots; used by the conflict-graph-ordering kernels.
#pragma once

#include "device.h"

namespace cce {

// A set of operation indices of one transaction (bit i <-> operation i),
// NW 64-bit words.  With L lanes per team, lane j's slot k holds operation
// j + k*L: for L < 64 every slot fits word 0, for L = 64 slot k is word k.
template <int NW>
struct OpSet {
  uint64_t w[NW];
  __device__ __forceinline__ static OpSet zero() {
    OpSet r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = 0;
    return r;
  }
  __device__ __forceinline__ OpSet operator|(const OpSet &o) const {
    OpSet r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = w[i] | o.w[i];
    return r;
  }
  __device__ __forceinline__ OpSet operator&(const OpSet &o) const {
    OpSet r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = w[i] & o.w[i];
    return r;
  }
  __device__ __forceinline__ OpSet operator~() const {
    OpSet r;
#pragma unroll
    for (int i = 0; i < NW; ++i) r.w[i] = ~w[i];
    return r;
  }
  __device__ __forceinline__ bool operator==(const OpSet &o) const {
    bool eq = true;
#pragma unroll
    for (int i = 0; i < NW; ++i) eq &= w[i] == o.w[i];
    return eq;
  }
  __device__ __forceinline__ bool test(uint32_t i) const {
    uint64_t x = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k)
      if ((int)(i >> 6) == k) x = w[k];
    return (x >> (i & 63)) & 1u;
  }
  // shift towards higher operation indices by s (0 < s < 64*NW)
  __device__ __forceinline__ OpSet up(int s) const {
    OpSet r;
    const int ws = s >> 6, bs = s & 63;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int j = i - ws;
      uint64_t v = j >= 0 ? (w[j] << bs) : 0;
      if (bs && j - 1 >= 0) v |= w[j - 1] >> (64 - bs);
      r.w[i] = v;
    }
    return r;
  }
  // shift towards lower operation indices by s
  __device__ __forceinline__ OpSet down(int s) const {
    OpSet r;
    const int ws = s >> 6, bs = s & 63;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int j = i + ws;
      uint64_t v = j < NW ? (w[j] >> bs) : 0;
      if (bs && j + 1 < NW) v |= w[j + 1] << (64 - bs);
      r.w[i] = v;
    }
    return r;
  }
};

// The team's set of slots for which p holds (team-uniform; all lanes of the
// wavefront must call it).
template <int L, int K, int NW>
__device__ __forceinline__ OpSet<NW> team_set(const Team<L> &t, const bool (&p)[K]) {
  OpSet<NW> r = OpSet<NW>::zero();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t b = ballot(p[k]);
    if constexpr (L == 64) {
      r.w[k] = b;
    } else {
      r.w[0] |= ((b >> t.tb) & ((1ull << L) - 1ull)) << (k * L);
    }
  }
  return r;
}

// Every operation of a row group inherits the bit of the group's first
// operation: x spreads to higher indices across followers (`fol`: bit i set
// when operation i continues the group of operation i-1).
template <int NW>
__device__ __forceinline__ OpSet<NW> spread_up(OpSet<NW> x, OpSet<NW> fol) {
#pragma unroll
  for (int s = 1; s < 64 * NW; s <<= 1) {
    x = x | (x.up(s) & fol);
    fol = fol & fol.up(s);
  }
  return x;
}

// A group's first operation collects the bits of its followers.
template <int NW>
__device__ __forceinline__ OpSet<NW> gather_down(OpSet<NW> x, OpSet<NW> fol) {
  OpSet<NW> nxt = fol.down(1);  // bit i: operation i+1 continues i's group
#pragma unroll
  for (int s = 1; s < 64 * NW; s <<= 1) {
    x = x | (x.down(s) & nxt);
    nxt = nxt & nxt.down(s);
  }
  return x;
}

}  // namespace cce
