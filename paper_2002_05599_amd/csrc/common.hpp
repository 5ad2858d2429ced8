// Device-side building blocks shared by the sorting kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "networks_gen.hpp"

namespace ss {

constexpr int kWave = 64;
constexpr int kMaxN = 256;
constexpr int kMaxNet = 16;

// Status codes written by kernels into the per-device status word
// (values match the public header).
constexpr int kStatusInval = -1;
constexpr int kStatusTooBig = -3;

// Keys are handled internally as unsigned words.  A signed key is mapped to
// unsigned by flipping its sign bit on load and back on store; this map is
// order-preserving, so the unsigned network sorts signed keys in
// two's-complement order.
template <class K> struct KeyTraits;
template <> struct KeyTraits<uint32_t> {
  static constexpr uint32_t kMax = 0xFFFFFFFFu;
  static constexpr uint32_t kSign = 0x80000000u;
};
template <> struct KeyTraits<uint64_t> {
  static constexpr uint64_t kMax = 0xFFFFFFFFFFFFFFFFull;
  static constexpr uint64_t kSign = 0x8000000000000000ull;
};

// Compare-exchange on keys alone (Section 2.1: the lower channel receives the
// smaller value).  For 32-bit keys this is one v_min_u32 and one v_max_u32;
// for 64-bit keys one 64-bit compare and four v_cndmask_b32.
__device__ __forceinline__ void cx(uint32_t& a, uint32_t& b) {
  uint32_t lo = min(a, b);
  uint32_t hi = max(a, b);
  a = lo;
  b = hi;
}
__device__ __forceinline__ void cx(uint64_t& a, uint64_t& b) {
  bool s = b < a;
  uint64_t lo = s ? b : a;
  uint64_t hi = s ? a : b;
  a = lo;
  b = hi;
}

// Compare-exchange of (key, value) pairs: swap exactly when the right key is
// strictly smaller (the paper's conditional swap), so equal keys never move
// their values.  This strictness is what lets padding channels filled with
// the maximum key stay in place (see pad_and_sort below).
template <class K>
__device__ __forceinline__ void cx_pair(K& a, K& b, uint32_t& va, uint32_t& vb) {
  bool s = b < a;
  K lo = s ? b : a;
  K hi = s ? a : b;
  uint32_t vlo = s ? vb : va;
  uint32_t vhi = s ? va : vb;
  a = lo;
  b = hi;
  va = vlo;
  vb = vhi;
}

template <class K, int N> struct KeyOp {
  K* r;
  __device__ __forceinline__ void operator()(int i, int j) { cx(r[i], r[j]); }
};
template <class K, int N> struct PairOp {
  K* r;
  uint32_t* v;
  __device__ __forceinline__ void operator()(int i, int j) { cx_pair(r[i], r[j], v[i], v[j]); }
};

// Sort N keys held in registers with the network of family F.
template <int F, int N, class K>
__device__ __forceinline__ void net_sort(K (&r)[N]) {
  KeyOp<K, N> op{r};
  Net<F, N>::run(op);
}
template <int F, int N, class K>
__device__ __forceinline__ void net_sort(K (&r)[N], uint32_t (&v)[N]) {
  PairOp<K, N> op{r, v};
  Net<F, N>::run(op);
}

// --- wave helpers ---------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t read_lane(uint32_t x, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)x);
}
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ uint64_t uniform(uint64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Records an error code in the device status word; the first error wins.
__device__ __forceinline__ void report(int* status, int code) {
  if (status) atomicCAS(status, 0, code);
}

}  // namespace ss
