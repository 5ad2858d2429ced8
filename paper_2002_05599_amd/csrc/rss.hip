// Register Sample Sort of many arrays of 17..256 keys in the fixed layout
// (array i at keys[i*stride, i*stride+n)).  A 256-thread work-group holds four
// waves; each wave sorts 64/G arrays at once, one per G-lane group, with
// G = 8, 16, 32 or 64 by the tuned bounds (at most 4 keys per lane).
#include "internal.hpp"
#include "large.hpp"
#include "rss.hpp"

namespace ss {

constexpr int kRssThreads = 256;
constexpr int kRssWaves = kRssThreads / kWave;

template <int F, class K, int G>
__global__ void __launch_bounds__(kRssThreads)
rss_fixed_kernel(K* __restrict__ keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, int k0, RssCfg cfg) {
  constexpr int kGroups = kWave / G;
  __shared__ GroupLds<K, 0, G> lds[kRssWaves * kGroups];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: keeps its uses scalar
  const int g = lane_id() / G;
  const int64_t arr = ((int64_t)blockIdx.x * kRssWaves + wave) * kGroups + g;
  const int m = arr < count ? n : 0;
  K* gk = keys + (arr < count ? arr * stride : 0);
  rss_group_sort<F, K, 0, G>(lds[wave * kGroups + g], gk, nullptr, m, flip, k0, cfg);
}

// The IS+SN alternative for 17..256 keys: one lane per array, insertion sort
// in global memory.
template <class K>
__global__ void __launch_bounds__(kRssThreads)
is_fixed_kernel(K* __restrict__ keys, int n, int64_t count, int64_t stride, KeyMap<K> flip) {
  const int64_t arr = (int64_t)blockIdx.x * kRssThreads + threadIdx.x;
  if (arr < count) insertion_sort_global<K, 0>(keys + arr * stride, nullptr, n, flip);
}

template <class K>
static hipError_t launch_is_fixed(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, hipStream_t s) {
  const int64_t blocks = (count + kRssThreads - 1) / kRssThreads;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(is_fixed_kernel<K>, dim3((unsigned)blocks), dim3(kRssThreads), 0, s, keys, n, count, stride,
                     flip);
  return hipGetLastError();
}

template <int F, class K, int G>
static hipError_t launch_rss_g(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, int k0,
                               RssCfg cfg, hipStream_t s) {
  constexpr int per_block = kRssWaves * (kWave / G);
  const int64_t blocks = (count + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((rss_fixed_kernel<F, K, G>), dim3((unsigned)blocks), dim3(kRssThreads), 0, s, keys, n,
                     count, stride, flip, k0, cfg);
  return hipGetLastError();
}

template <int F, class K>
static hipError_t launch_rss_f(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, hipStream_t s) {
  const Tuning t = tuning(sizeof(K));
  const RssCfg cfg{t.rss_level_cap, t.rss_oversample, t.rss_finish};
  // the same lane-group mapping as the segmented size classes
  if (n <= t.rss_bound_tiny) return launch_rss_g<F, K, 8>(keys, n, count, stride, flip, 8, cfg, s);
  if (n <= t.rss_bound_small) return launch_rss_g<F, K, 16>(keys, n, count, stride, flip, t.rss_k[0], cfg, s);
  if (n <= t.rss_bound_mid) return launch_rss_g<F, K, 32>(keys, n, count, stride, flip, t.rss_k[1], cfg, s);
  return launch_rss_g<F, K, 64>(keys, n, count, stride, flip, t.rss_k[2], cfg, s);
}

hipError_t launch_rss_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                                int* status, hipStream_t s) {
  (void)status;
  if (n < 17 || n > kMaxN) return hipErrorInvalidValue;
  if (tuning(sizeof(*keys)).large_sort == 1) return launch_is_fixed(keys, n, count, stride, flip, s);
  switch (tuning(sizeof(*keys)).family) {
    case 1: return launch_rss_f<1>(keys, n, count, stride, flip, s);
    case kFamilyInsertion: return launch_rss_f<kFamilyInsertion>(keys, n, count, stride, flip, s);
    default: return launch_rss_f<0>(keys, n, count, stride, flip, s);
  }
}
hipError_t launch_rss_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                                int* status, hipStream_t s) {
  (void)status;
  if (n < 17 || n > kMaxN) return hipErrorInvalidValue;
  if (tuning(sizeof(*keys)).large_sort == 1) return launch_is_fixed(keys, n, count, stride, flip, s);
  switch (tuning(sizeof(*keys)).family) {
    case 1: return launch_rss_f<1>(keys, n, count, stride, flip, s);
    case kFamilyInsertion: return launch_rss_f<kFamilyInsertion>(keys, n, count, stride, flip, s);
    default: return launch_rss_f<0>(keys, n, count, stride, flip, s);
  }
}

// Arrays of 257..4096 keys: one work-group per array (large.hpp); with
// large_sort = 1, insertion sort by one lane per array (IS+SN).
template <int F, class K>
__global__ void __launch_bounds__(kLargeThreads)
large_fixed_kernel(K* __restrict__ keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, int k0, RssCfg cfg) {
  extern __shared__ __attribute__((aligned(16))) unsigned char large_lds[];
  for (int64_t arr = blockIdx.x; arr < count; arr += gridDim.x)
    large_sort<F, K, 0>(large_lds, keys + arr * stride, nullptr, n, flip, k0, cfg);
}

template <int F, class K>
static hipError_t launch_large_f(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, hipStream_t s) {
  const Tuning t = tuning(sizeof(K));
  constexpr size_t kLds = LargeLds<K, 0>::kBytes;
  static const hipError_t attr = allow_dynamic_lds(large_fixed_kernel<F, K>, kLds);
  if (attr != hipSuccess) return attr;
  const int64_t blocks = count < (1 << 20) ? count : (1 << 20);
  hipLaunchKernelGGL((large_fixed_kernel<F, K>), dim3((unsigned)blocks), dim3(kLargeThreads), kLds, s, keys, n,
                     count, stride, flip, t.rss_k[2], RssCfg{t.rss_level_cap, t.rss_oversample, t.rss_finish});
  return hipGetLastError();
}

template <class K>
static hipError_t launch_large_any(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, hipStream_t s) {
  if (n <= kMaxN || n > kMaxLargeN) return hipErrorInvalidValue;
  if (tuning(sizeof(*keys)).large_sort == 1) return launch_is_fixed(keys, n, count, stride, flip, s);
  switch (tuning(sizeof(*keys)).family) {
    case 1: return launch_large_f<1>(keys, n, count, stride, flip, s);
    case kFamilyInsertion: return launch_large_f<kFamilyInsertion>(keys, n, count, stride, flip, s);
    default: return launch_large_f<0>(keys, n, count, stride, flip, s);
  }
}

hipError_t launch_large_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                                  hipStream_t s) {
  return launch_large_any(keys, n, count, stride, flip, s);
}
hipError_t launch_large_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                                  hipStream_t s) {
  return launch_large_any(keys, n, count, stride, flip, s);
}

}  // namespace ss
