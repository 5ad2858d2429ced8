// Arrays of 257..4096 keys: one 256-thread work-group per array.
//
// Section 5 names merge sort with merging networks as the way to build on the
// small sorters for larger inputs.  Here the array of m keys is cut into 4r
// runs of equal length (r = ceil(m / 1024), the length rounded up to a
// multiple of 8, at most 256 keys), so that each of the four waves sorts r
// runs; each wave sorts its runs with Register Sample Sort (the same G = 64
// group sort as the 129..256-key class), and the sorted runs are then merged
// pairwise in LDS, doubling the run length each round (at most four rounds
// for 4096 keys).  In a merge round every thread produces the same number P
// of consecutive outputs, the smallest power of two that lets the 256 threads
// cover the array (2 for up to 512 keys, 16 for 4096).  It finds where its
// first output's diagonal crosses the two runs by a binary search (merge
// path; ties are taken from the left run first) and then merges its items
// sequentially, holding the next key of each run in registers so that a step
// reads one key from LDS.  (Reading both runs' next P keys at once and
// ordering them with a bitonic merge in registers was measured no faster.)
//
// LDS holds two buffers of kMaxLargeN items (keys as order-preserving words,
// then payloads).  The second buffer also holds the waves' Register Sample
// Sort state while the runs are sorted; it is free again for the merges.
#pragma once

#include "rss.hpp"

namespace ss {

constexpr int kLargeThreads = 256;
constexpr int kMaxLargeN = 4096;
constexpr int kRunN = 256;                               // most keys per run (one G = 64 group)
constexpr int kMergePerMax = kMaxLargeN / kLargeThreads;  // merge outputs per thread at 4096 keys

template <class K, int V> struct LargeLds {
  static constexpr size_t kKeyBytes = (size_t)kMaxLargeN * sizeof(K);
  static constexpr size_t kValBytes = V ? (size_t)kMaxLargeN * sizeof(Pay<V>) : 0;
  static constexpr size_t kBufBytes = kKeyBytes + kValBytes;
  static constexpr size_t kGroupBytes = (kLargeThreads / kWave) * sizeof(GroupLds<K, V, 64>);
  // the second buffer also holds the run sorts' state
  static constexpr size_t kBytes = kBufBytes + (kGroupBytes > kBufBytes ? kGroupBytes : kBufBytes);
};

// One thread's share of a merge round: outputs out0 .. out0 + P - 1 of the
// merge of the run pair that holds them (P divides 2L, so a share never spans
// two pairs).  sk/sv hold runs of L sorted words, dk/dv receive runs of 2L.
template <int P, class K, int V>
__device__ __forceinline__ void merge_block(const K* sk, const Pay<V>* sv, K* dk, Pay<V>* dv, int m, int L) {
  const int out0 = (int)threadIdx.x * P;
  if (out0 >= m) return;
  const int a0 = (out0 / (2 * L)) * (2 * L);
  const int la = min(L, m - a0);  // >= 1
  const int b0 = a0 + la;
  const int lb = min(L, m - b0);  // 0 for a last run without partner
  const int d = out0 - a0;
  // merge path: i keys of the left run among the first d outputs
  int lo = max(0, d - lb), hi = min(d, la);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sk[a0 + mid] <= sk[b0 + d - 1 - mid])
      lo = mid + 1;
    else
      hi = mid;
  }
  int i = lo, j = d - lo;
  const int n_out = min(P, la + lb - d);
  // the next key of each run (la >= 1; a key read past a run's end is never used)
  K ka = sk[a0 + min(i, la - 1)];
  K kb = lb > 0 ? sk[b0 + min(j, lb - 1)] : K(0);
  for (int e = 0; e < n_out; ++e) {
    const bool take_a = i < la && (j >= lb || ka <= kb);
    const int src = take_a ? a0 + i : b0 + j;
    dk[out0 + e] = take_a ? ka : kb;
    if constexpr (V) dv[out0 + e] = sv[src];
    i += take_a ? 1 : 0;
    j += take_a ? 0 : 1;
    // refill from the run that gave its key
    const K kn = sk[take_a ? a0 + min(i, la - 1) : b0 + min(j, max(lb - 1, 0))];
    ka = take_a ? kn : ka;
    kb = take_a ? kb : kn;
  }
}

// Sorts the m (<= kMaxLargeN) keys at gk (and payloads at gv) with the whole
// work-group; every thread of the work-group must call this.
template <int F, class K, int V>
__device__ __forceinline__ void large_sort(unsigned char* lds, K* gk, Pay<V>* gv, int m, KeyMap<K> flip, int k0,
                                           RssCfg cfg) {
  using LL = LargeLds<K, V>;
  using VT = Pay<V>;
  K* key_buf[2] = {reinterpret_cast<K*>(lds), reinterpret_cast<K*>(lds + LL::kBufBytes)};
  VT* val_buf[2] = {reinterpret_cast<VT*>(lds + LL::kKeyBytes),
                    reinterpret_cast<VT*>(lds + LL::kBufBytes + LL::kKeyBytes)};
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  auto* group = reinterpret_cast<GroupLds<K, V, 64>*>(lds + LL::kBufBytes) + wave;

  // 4 rr runs of at most kRunN keys, a multiple of 8 each (so that 2 run is a
  // multiple of the merge's outputs per thread), run r by wave r mod 4
  constexpr int kWaves = kLargeThreads / kWave;
  const int rr = (m + kWaves * kRunN - 1) / (kWaves * kRunN);
  const int run = (((m + kWaves * rr - 1) / (kWaves * rr)) + 7) & ~7;
  const int nruns = (m + run - 1) / run;
  for (int r = wave; r < nruns; r += kWaves) {
    const int lo = r * run;
    const int len = min(run, m - lo);
    rss_group_load(*group, gk + lo, V ? gv + lo : nullptr, len, flip);
    wave_lds_sync();
    rss_group_sort_lds<F>(*group, len, k0, cfg);
    for (int i = lane; i < len; i += kWave) {
      key_buf[0][lo + i] = group->key[i];
      if constexpr (V) val_buf[0][lo + i] = group->val[i];
    }
    wave_lds_sync();
  }
  __syncthreads();

  // merge rounds: runs of length L in buffer `cur` -> runs of 2L in the other;
  // P outputs per thread, a power of two of at most 16, so that it divides 2L
  // (a multiple of 16)
  const int per = m <= 512 ? 2 : (m <= 1024 ? 4 : (m <= 2048 ? 8 : kMergePerMax));
  int cur = 0;
  for (int L = run; L < m; L *= 2) {
    const K* sk = key_buf[cur];
    const VT* sv = val_buf[cur];
    K* dk = key_buf[cur ^ 1];
    VT* dv = val_buf[cur ^ 1];
    switch (per) {
      case 2: merge_block<2, K, V>(sk, sv, dk, dv, m, L); break;
      case 4: merge_block<4, K, V>(sk, sv, dk, dv, m, L); break;
      case 8: merge_block<8, K, V>(sk, sv, dk, dv, m, L); break;
      default: merge_block<kMergePerMax, K, V>(sk, sv, dk, dv, m, L); break;
    }
    __syncthreads();
    cur ^= 1;
  }

  // store, mapping the words back to keys
  for (int i = (int)threadIdx.x; i < m; i += kLargeThreads) {
    gk[i] = flip.dec(key_buf[cur][i]);
    if constexpr (V) gv[i] = val_buf[cur][i];
  }
  __syncthreads();
}

// Lets a kernel use `bytes` of dynamic LDS (above the default limit of the
// launch); called once per kernel before its first launch.
template <class Kernel>
inline hipError_t allow_dynamic_lds(Kernel kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace ss
