// Order-preserving map of every key type onto unsigned words of its width.
// The sorting kernels compare unsigned words; a key is mapped on load and
// mapped back on store:
//   unsigned integers  unchanged;
//   signed integers    the sign bit is flipped (two's-complement order);
//   IEEE floats        a negative value has every bit flipped, a positive one
//                      only its sign bit, so that the unsigned order of the
//                      words is the IEEE 754 totalOrder of the floats:
//                      -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN.
// In one formula: word = key ^ (flip | (top(key) & neg)), where top(x) is all
// ones when the top bit of x is set; neg = all ones for floats, 0 otherwise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ss {

template <class K> struct KeyMap {
  K flip;  // bits flipped in every key
  K neg;   // bits flipped in addition in keys whose top bit is set
  __host__ __device__ __forceinline__ static K top(K x) {
    using S = typename std::conditional<sizeof(K) == 8, int64_t, int32_t>::type;
    return (K)((S)x >> (8 * sizeof(K) - 1));
  }
  __host__ __device__ __forceinline__ K enc(K x) const { return x ^ (flip | (top(x) & neg)); }
  // a word's top bit is clear exactly when its key was a negative float
  __host__ __device__ __forceinline__ K dec(K y) const { return y ^ (flip | (top(~y) & neg)); }

  // The same maps over a whole register array, choosing the form once: the
  // integer keys (neg == 0, a launch-wide value) take a single XOR per key.
  template <int N>
  __device__ __forceinline__ void enc_all(K (&r)[N]) const {
    if (neg == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] ^= flip;
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] = enc(r[j]);
    }
  }
  template <int N>
  __device__ __forceinline__ void dec_all(K (&r)[N]) const {
    if (neg == 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] ^= flip;
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] = dec(r[j]);
    }
  }
};

template <class K> constexpr KeyMap<K> kUnsignedMap{K(0), K(0)};
template <class K> constexpr KeyMap<K> kSignedMap{K(K(1) << (8 * sizeof(K) - 1)), K(0)};
template <class K> constexpr KeyMap<K> kFloatMap{K(K(1) << (8 * sizeof(K) - 1)), K(~K(0))};

}  // namespace ss
