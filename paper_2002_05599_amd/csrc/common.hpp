// Device-side building blocks shared by the sorting kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "keymap.hpp"
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
// Payload word for a payload of VB bytes per key (VB = 0: no payload; the
// type is then a placeholder that is never read or written).
template <int VB> struct PayloadWord { using type = uint32_t; };
template <> struct PayloadWord<8> { using type = uint64_t; };
template <int VB> using Pay = typename PayloadWord<VB>::type;

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
template <class K, class VT>
__device__ __forceinline__ void cx_pair(K& a, K& b, VT& va, VT& vb) {
  bool s = b < a;
  K lo = s ? b : a;
  K hi = s ? a : b;
  VT vlo = s ? vb : va;
  VT vhi = s ? va : vb;
  a = lo;
  b = hi;
  va = vlo;
  vb = vhi;
}

template <class K, int N> struct KeyOp {
  K* r;
  __device__ __forceinline__ void operator()(int i, int j) { cx(r[i], r[j]); }
};
template <class K, int N, class VT> struct PairOp {
  K* r;
  VT* v;
  __device__ __forceinline__ void operator()(int i, int j) { cx_pair(r[i], r[j], v[i], v[j]); }
};

// "Family" 2 is not a network: the textbook insertion sort the paper measures
// the networks against ("IS Def", Section 4.2), as the baseline variant.
constexpr int kFamilyInsertion = 2;

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Insertion sort of N keys (and values) held in registers: key i is moved left
// past every larger key (strict compare, so it is stable), as in the textbook
// loop.  Channel indices are compile-time constants (fully unrolled, no
// dynamic register indexing); the inner loop ends as soon as no lane of the
// wave is still shifting, so an already sorted input costs one compare per
// key, as on the CPU, and the cost of a wave is that of its slowest lane.
template <int N, class K, bool V, class VT>
__device__ __forceinline__ void insertion_sort_regs(K (&r)[N], VT* v) {
#pragma unroll
  for (int i = 1; i < N; ++i) {
    const K x = r[i];
    VT xv = 0;
    if constexpr (V) xv = v[i];
    bool go = true;  // this lane has not placed x yet
#pragma unroll
    for (int j = i - 1; j >= 0; --j) {
      if (!wave_any(go)) break;
      const bool shift = go && r[j] > x;
      // shifting: r[j] moves up; stopping here: x lands at j + 1
      r[j + 1] = shift ? r[j] : (go ? x : r[j + 1]);
      if constexpr (V) v[j + 1] = shift ? v[j] : (go ? xv : v[j + 1]);
      go = shift;
    }
    if (go) {
      r[0] = x;
      if constexpr (V) v[0] = xv;
    }
  }
}

// Textbook insertion sort of one array of n keys (and values) in place in
// global memory, by one lane: the larger-sets half of the paper's IS+SN
// hybrid (Section 4.6: networks up to 16 keys, insertion sort above).  Keys
// are compared as their order-preserving words (flip.enc).
template <class K, int V>
__device__ __forceinline__ void insertion_sort_global(K* p, Pay<V>* pv, int n, KeyMap<K> flip) {
  for (int i = 1; i < n; ++i) {
    const K xs = p[i];
    const K x = flip.enc(xs);
    Pay<V> xv = 0;
    if constexpr (V) xv = pv[i];
    int j = i - 1;
    while (j >= 0) {
      const K ys = p[j];
      if (!(flip.enc(ys) > x)) break;
      p[j + 1] = ys;
      if constexpr (V) pv[j + 1] = pv[j];
      --j;
    }
    p[j + 1] = xs;
    if constexpr (V) pv[j + 1] = xv;
  }
}

// Sort N keys held in registers with the network of family F (or, for
// kFamilyInsertion, with insertion sort).
template <int F, int N, class K>
__device__ __forceinline__ void net_sort(K (&r)[N]) {
  if constexpr (F == kFamilyInsertion) {
    insertion_sort_regs<N, K, false, uint32_t>(r, nullptr);
  } else {
    KeyOp<K, N> op{r};
    Net<F, N>::run(op);
  }
}
template <int F, int N, class K, class VT>
__device__ __forceinline__ void net_sort(K (&r)[N], VT (&v)[N]) {
  if constexpr (F == kFamilyInsertion) {
    insertion_sort_regs<N, K, true, VT>(r, v);
  } else {
    PairOp<K, N, VT> op{r, v};
    Net<F, N>::run(op);
  }
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
