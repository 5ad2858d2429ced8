// Segmented (CSR) sorting of ragged batches: segment i is
// keys[offsets[i], offsets[i+1]), sizes 0..256, with an optional uint32
// payload permuted with the keys.
//
// Section 5 proposes, as future work, to group the base cases by their size
// and to sort each group of equally sized subproblems together.  That is what
// happens here, entirely on the device:
//
//   count    each block histograms the size classes of its segments
//   scan     one block turns the per-block histograms into class totals,
//            class start offsets and per-block output bases; zeroes the
//            claim counters
//   scatter  each block writes its segment ids into the class lists (segment
//            ids grouped by class; no contended atomics)
//   sort     persistent kernels, by default one per kind: the network
//            classes (one segment per lane, the network of exactly that size
//            in registers, 64-segment tiles; or, tuned, every network size in
//            batch order, each tile staged through LDS as one run), then each
//            RSS class (Register Sample Sort with 8-, 16-, 32- or 64-lane
//            groups, rss.hpp).  Work is split into 8 partitions, one
//            per XCD (blockIdx mod 8), each with its own claim counter; waves
//            take their share round-robin and claim the remainder in small
//            pieces at the end, so they finish together.  A single kernel for
//            every class is kept as a tuning choice.
//
// Size classes: 0..14 = sizes 2..16; 15..18 = the RSS classes of 8-, 16-,
// 32- and 64-lane groups (17..bt, ..bs, ..bm, ..256 keys for the tuned bounds
// bt <= bs <= bm; by default 17..32, 33..64, 65..128, 129..256); 19 =
// 257..4096 (one work-group per segment: Register Sample Sort of runs of 256
// keys, then merge rounds in LDS, large.hpp).  Sizes 0 and 1 need no work.
// A segment longer than 4096 keys or with a negative size is skipped and
// flagged in the status word.
//
// Modes: the binning and persistent kernels replayed from a cached hipGraph
// (built once per key type / payload / network family / kernel split; each
// call only rewrites the kernel arguments of its nodes), the same kernels
// launched directly, or the "plain" baseline: the binning, a copy of the
// class counts to the host, then one ordinary launch per non-empty class.
#pragma once

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "large.hpp"
#include "rss.hpp"

namespace ss {

constexpr int kClasses = 20;       // size classes of the binning
constexpr int kTiledClasses = 19;  // classes sorted in wave-sized tiles (networks, RSS)
constexpr int kLargeClass = 19;    // 257..4096 keys: one work-group per segment
constexpr int kNetClasses = 15;
constexpr int kRssClasses = 4;     // 15..18: 8-, 16-, 32-, 64-lane groups

// Lanes per array of RSS class c (15..18), and arrays per wave.
__host__ __device__ constexpr int rss_group(int c) { return 8 << (c - kNetClasses); }
__host__ __device__ constexpr int class_groups(int c) { return c < kNetClasses ? 1 : kWave / rss_group(c); }
constexpr int kBinThreads = 256;
constexpr int kBinItems = 4;                       // segments per thread per chunk
constexpr int kBinChunk = kBinThreads * kBinItems;  // segments per block iteration
constexpr int kBinBlocks = 1024;                   // fixed grid of count/scatter
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;

// ctrl layout (uint32 words)
constexpr int kCtrlCount = 0;        // [kClasses] segments per class
constexpr int kCtrlStart = 32;       // [kClasses] start of each class list
constexpr int kCtrlTile = 128;       // tile counters: kind set k, partition p at kCtrlTile + (8k + p) * 32
constexpr int kTileParts = 8;        // counter partitions (one 128-byte line each)
constexpr int kCtrlWords = kCtrlTile + 7 * kTileParts * 32;  // 7 kind sets
static_assert(kCtrlWords * 4 <= (int)kSegCtrlBytes && kBinBlocks * kClasses * 4 == (int)kSegHistBytes,
              "the binning's buffers have the sizes the other units assume");

// bt, bs, bm: the largest sizes given to 8-, 16- and 32-lane RSS groups
// (tuned: bt in 16..32, bs in bt..64, bm in bs..128; a G-lane group holds up
// to 4G keys).
__device__ __forceinline__ int size_class(int sz, int bt, int bs, int bm) {
  if (sz < 2) return sz >= 0 ? -1 : -3;  // -1: nothing to do, -3: bad offsets
  if (sz <= 16) return sz - 2;
  if (sz <= bt) return 15;
  if (sz <= bs) return 16;
  if (sz <= bm) return 17;
  if (sz <= kMaxN) return 18;
  if (sz <= kMaxLargeN) return kLargeClass;
  return -2;  // too big
}

// Rounds of RSS lane groups per tile for class c: at most `rounds`, and few
// enough that the class still has about `tpw` tiles per resident wave (a
// class with few segments would otherwise leave most waves idle).  The
// persistent kernels balance their tails dynamically and do best with fewer,
// larger tiles (kPersistTpw); one launch per class relies on the hardware
// dispatcher and does best with more (kPlainTpw).
constexpr int kPersistTpw = 4;
constexpr int kPlainTpw = 8;
__host__ __device__ __forceinline__ int class_rounds(int c, int count, int rounds, int waves, int tpw) {
  if (c < kNetClasses) return 1;
  const int per = class_groups(c) * waves * tpw;
  const int r = count / (per > 0 ? per : 1);
  return r < 1 ? 1 : (r > rounds ? rounds : r);
}

// Tile size (segments) of a class; rounds = RSS group rounds per tile.
__host__ __device__ __forceinline__ int class_tile(int c, int rounds) {
  if (c < kNetClasses) return kWave;
  return class_groups(c) * rounds;
}

// Classes in the order the persistent kernel hands out tiles: the RSS
// classes largest first, then the network classes.
__host__ __device__ __forceinline__ int class_at(int order) {
  return order < kRssClasses ? kNetClasses + kRssClasses - 1 - order : kNetClasses - 1 - (order - kRssClasses);
}

// --- binning kernels (segmented_common.hip) -----------------------------------

__global__ void seg_count_kernel(const int32_t* __restrict__ offsets, int32_t nseg,
                                 uint32_t* __restrict__ blockhist, int* status, int bins);
__global__ void seg_scan_kernel(uint32_t* __restrict__ blockhist, int nblocks, uint32_t* __restrict__ ctrl);
__global__ void seg_scatter_kernel(const int32_t* __restrict__ offsets, int32_t nseg,
                                   const uint32_t* __restrict__ blockbase, const uint32_t* __restrict__ ctrl,
                                   int32_t* __restrict__ ids, int bins);

// The binning's parameters in one word: bit 0 = every network size goes to
// class 0, whose segments are then sorted in batch order (see
// net_tile_staged); bits 8..15, 16..23 and 24..31 = the RSS class bounds bs,
// bm and bt.
__host__ __device__ __forceinline__ int pack_bins(int mix, int bt, int bs, int bm) {
  return (mix ? 1 : 0) | (bs << 8) | (bm << 16) | (bt << 24);
}
__device__ __forceinline__ int bin_class(int sz, int bins) {
  const int c = size_class(sz, (bins >> 24) & 0xFF, (bins >> 8) & 0xFF, (bins >> 16) & 0xFF);
  return ((bins & 1) && c > 0 && c < kNetClasses) ? 0 : c;
}

// --- tile handlers -----------------------------------------------------------

template <int F, int N, class K, int V>
__device__ __forceinline__ void net_tile(K* __restrict__ keys, Pay<V>* __restrict__ vals,
                                         const int32_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                                         int list, int count, int first, KeyMap<K> flip) {
  const int j = first + lane_id();
  if (j >= count) return;
  const int seg = ids[list + j];
  K* p = keys + offsets[seg];
  K r[N];
  Pay<V> v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = flip.enc(p[i]);
  if constexpr (V) {
    Pay<V>* pv = vals + offsets[seg];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = pv[i];
    net_sort<F, N>(r, v);
#pragma unroll
    for (int i = 0; i < N; ++i) pv[i] = v[i];
  } else {
    net_sort<F, N>(r);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = flip.dec(r[i]);
}

template <int F, class K, int V>
__device__ __forceinline__ void net_tile_dispatch(int n, K* keys, Pay<V>* vals, const int32_t* offsets,
                                                  const int32_t* ids, int list, int count, int first, KeyMap<K> flip) {
  switch (n) {
    case 2: net_tile<F, 2, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 3: net_tile<F, 3, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 4: net_tile<F, 4, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 5: net_tile<F, 5, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 6: net_tile<F, 6, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 7: net_tile<F, 7, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 8: net_tile<F, 8, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 9: net_tile<F, 9, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 10: net_tile<F, 10, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 11: net_tile<F, 11, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 12: net_tile<F, 12, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 13: net_tile<F, 13, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 14: net_tile<F, 14, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    case 15: net_tile<F, 15, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
    default: net_tile<F, 16, K, V>(keys, vals, offsets, ids, list, count, first, flip); break;
  }
}

// One segment of n <= N keys in the channels 0..n-1 of an N-key network;
// channels n.. hold the maximum key, which the strict compare-exchange never
// moves, so channels 0..n-1 end sorted.
template <int F, int N, class K, int V>
__device__ __forceinline__ void net_sort_padded(K* __restrict__ p, Pay<V>* __restrict__ pv, int n, KeyMap<K> flip) {
  K r[N];
  Pay<V> v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = i < n ? flip.enc(p[i]) : KeyTraits<K>::kMax;
  if constexpr (V) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = i < n ? pv[i] : Pay<V>(0);
    net_sort<F, N>(r, v);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i < n) pv[i] = v[i];
  } else {
    net_sort<F, N>(r);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < n) p[i] = flip.dec(r[i]);
}

// A tile of 64 segments of 2..16 keys of any sizes, in batch order (the
// class-0 list when the binning mixes the network sizes): one segment per
// lane, every lane running the network of the wave's largest segment.
// Segments that are neighbours in memory are then read by the same wave at
// the same time and share their cache lines, where per-size classes would
// read each line once per class that touches it.
template <int F, class K, int V>
__device__ __forceinline__ void net_tile_mixed(K* keys, Pay<V>* vals, const int32_t* __restrict__ offsets,
                                               const int32_t* __restrict__ ids, int list, int count, int first,
                                               KeyMap<K> flip) {
  const int j = first + lane_id();
  int lo = 0, n = 0;
  if (j < count) {
    const int seg = ids[list + j];
    lo = offsets[seg];
    n = offsets[seg + 1] - lo;
  }
  const int nmax = (int)wave_max((uint32_t)n);
  K* p = keys + lo;
  Pay<V>* pv = V ? vals + lo : nullptr;
  switch (nmax) {
    case 2: net_sort_padded<F, 2, K, V>(p, pv, n, flip); break;
    case 3: net_sort_padded<F, 3, K, V>(p, pv, n, flip); break;
    case 4: net_sort_padded<F, 4, K, V>(p, pv, n, flip); break;
    case 5: net_sort_padded<F, 5, K, V>(p, pv, n, flip); break;
    case 6: net_sort_padded<F, 6, K, V>(p, pv, n, flip); break;
    case 7: net_sort_padded<F, 7, K, V>(p, pv, n, flip); break;
    case 8: net_sort_padded<F, 8, K, V>(p, pv, n, flip); break;
    case 9: net_sort_padded<F, 9, K, V>(p, pv, n, flip); break;
    case 10: net_sort_padded<F, 10, K, V>(p, pv, n, flip); break;
    case 11: net_sort_padded<F, 11, K, V>(p, pv, n, flip); break;
    case 12: net_sort_padded<F, 12, K, V>(p, pv, n, flip); break;
    case 13: net_sort_padded<F, 13, K, V>(p, pv, n, flip); break;
    case 14: net_sort_padded<F, 14, K, V>(p, pv, n, flip); break;
    case 15: net_sort_padded<F, 15, K, V>(p, pv, n, flip); break;
    default: net_sort_padded<F, 16, K, V>(p, pv, n, flip); break;
  }
}

// LDS of one wave for a staged tile of mixed network sizes: the tile's keys
// (and payloads) as one run of at most 64 x 16 elements plus a sink entry, the
// segment of each element, and each segment's start in memory and in the run.
constexpr int kNetRun = kWave * kMaxNet;
template <class K, int V> struct NetLds {
  K key[kNetRun + 1];
  Pay<V> val[V ? kNetRun + 1 : 1];
  int32_t start[kWave];
  int32_t pre[kWave];
  uint8_t owner[kNetRun];
};

// A tile of 64 consecutive segments of 2..16 keys in batch order (the class-0
// list when the binning mixes the network sizes), staged through LDS: the
// wave reads the tile's segments as one run of elements -- element e of their
// concatenation belongs to segment owner[e] -- so each load instruction covers
// 64 consecutive elements of neighbouring segments instead of one element of
// 64 segments; each lane then sorts its own segment from LDS with the network
// of the tile's largest segment (channels past the segment hold the maximum
// key) and the run is stored back the same way.
template <int N, int F, class K, int V>
__device__ __forceinline__ void net_sort_run(NetLds<K, V>& S, int pre, int n) {
  K r[N];
  Pay<V> v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = i < n ? S.key[pre + i] : KeyTraits<K>::kMax;
  if constexpr (V) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = S.val[i < n ? pre + i : kNetRun];
    net_sort<F, N>(r, v);
  } else {
    net_sort<F, N>(r);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int d = i < n ? pre + i : kNetRun;  // the sink
    S.key[d] = r[i];
    if constexpr (V) S.val[d] = v[i];
  }
}

template <int F, class K, int V>
__device__ __forceinline__ void net_tile_staged(unsigned char* wave_lds, K* keys, Pay<V>* vals,
                                                const int32_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                                                int list, int count, int first, KeyMap<K> flip) {
  auto& S = *reinterpret_cast<NetLds<K, V>*>(wave_lds);
  const int lane = lane_id();
  const int j = first + lane;
  int lo = 0, n = 0;
  if (j < count) {
    const int seg = ids[list + j];
    lo = offsets[seg];
    n = offsets[seg + 1] - lo;
  }
  const int incl = (int)segment_scan<kWave>((uint32_t)n);
  const int pre = incl - n;
  const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
  const int nmax = (int)wave_max((uint32_t)n);
  S.start[lane] = lo;
  S.pre[lane] = pre;
  for (int i = 0; i < n; ++i) S.owner[pre + i] = (uint8_t)lane;
  wave_lds_sync();
  // the run in: every element's load is issued before any is written to LDS
  K x[kMaxNet];
  Pay<V> y[kMaxNet];
#pragma unroll
  for (int t = 0; t < kMaxNet; ++t) {
    const int e = lane + kWave * t;
    if (e < total) {
      const int o = S.owner[e];
      const int a = S.start[o] + (e - S.pre[o]);
      x[t] = keys[a];
      if constexpr (V) y[t] = vals[a];
    }
  }
#pragma unroll
  for (int t = 0; t < kMaxNet; ++t) {
    const int e = lane + kWave * t;
    if (e < total) {
      S.key[e] = flip.enc(x[t]);
      if constexpr (V) S.val[e] = y[t];
    }
  }
  wave_lds_sync();
  switch (nmax) {
    case 0: case 1: break;
    case 2: net_sort_run<2, F>(S, pre, n); break;
    case 3: net_sort_run<3, F>(S, pre, n); break;
    case 4: net_sort_run<4, F>(S, pre, n); break;
    case 5: net_sort_run<5, F>(S, pre, n); break;
    case 6: net_sort_run<6, F>(S, pre, n); break;
    case 7: net_sort_run<7, F>(S, pre, n); break;
    case 8: net_sort_run<8, F>(S, pre, n); break;
    case 9: net_sort_run<9, F>(S, pre, n); break;
    case 10: net_sort_run<10, F>(S, pre, n); break;
    case 11: net_sort_run<11, F>(S, pre, n); break;
    case 12: net_sort_run<12, F>(S, pre, n); break;
    case 13: net_sort_run<13, F>(S, pre, n); break;
    case 14: net_sort_run<14, F>(S, pre, n); break;
    case 15: net_sort_run<15, F>(S, pre, n); break;
    default: net_sort_run<16, F>(S, pre, n); break;
  }
  wave_lds_sync();
  // the run out
#pragma unroll
  for (int t = 0; t < kMaxNet; ++t) {
    const int e = lane + kWave * t;
    if (e < total) {
      const int o = S.owner[e];
      const int a = S.start[o] + (e - S.pre[o]);
      keys[a] = flip.dec(S.key[e]);
      if constexpr (V) vals[a] = S.val[e];
    }
  }
  wave_lds_sync();
}

// Per-wave LDS big enough for any RSS group layout of this key type.
template <class K, int V> struct WaveLds {
  static constexpr size_t kBytes8 = 8 * sizeof(GroupLds<K, V, 8>);
  static constexpr size_t kBytes16 = 4 * sizeof(GroupLds<K, V, 16>);
  static constexpr size_t kBytes32 = 2 * sizeof(GroupLds<K, V, 32>);
  static constexpr size_t kBytes64 = sizeof(GroupLds<K, V, 64>);
  static constexpr size_t kBytesA = kBytes8 > kBytes16 ? kBytes8 : kBytes16;
  static constexpr size_t kBytesB = kBytes32 > kBytes64 ? kBytes32 : kBytes64;
  static constexpr size_t kBytes = kBytesA > kBytesB ? kBytesA : kBytesB;
};

// One tile: `rounds` rounds of kWave/G arrays (one per G-lane group).  The
// segment bounds of up to 64 arrays are fetched at once (one per lane) and
// handed to the groups with lane permutes, and the next round's keys are
// loaded into registers before the current round is sorted, so the sort
// hides the load latency.
template <int F, class K, int V, int G>
__device__ __forceinline__ void rss_tile(unsigned char* wave_lds, K* keys, Pay<V>* vals,
                                         const int32_t* __restrict__ offsets, const int32_t* __restrict__ ids,
                                         int list, int count, int first, int rounds, KeyMap<K> flip, int k0,
                                         RssCfg cfg) {
  constexpr int kGroups = kWave / G;
  auto* L = reinterpret_cast<GroupLds<K, V, G>*>(wave_lds);
  const int lane = lane_id();
  const int g = lane / G;
  const int narr = rounds * kGroups;
  int meta_lo = 0, meta_m = 0;  // lane l: bounds of array a0 + l of the tile
  auto bounds = [&](int r, int& lo, int& m) __attribute__((always_inline)) {
    const int a0 = r * kGroups;
    if ((a0 & (kWave - 1)) == 0) {
      const int a = a0 + lane;
      const int j = first + a;
      meta_lo = 0;
      meta_m = 0;
      if (a < narr && j < count) {
        const int seg = ids[list + j];
        meta_lo = offsets[seg];
        meta_m = offsets[seg + 1] - meta_lo;
      }
    }
    const int src = (a0 & (kWave - 1)) + g;
    if constexpr (G == kWave) {
      // one array per wave: its bounds are wave-uniform (scalar registers)
      lo = __builtin_amdgcn_readlane(meta_lo, src);
      m = __builtin_amdgcn_readlane(meta_m, src);
    } else {
      lo = (int)read_lane((uint32_t)meta_lo, src);
      m = (int)read_lane((uint32_t)meta_m, src);
    }
  };
  const int gl = lane % G;
  K nk[4];
  Pay<V> nv[4];
  auto fetch = [&](int lo, int m) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      if (i < m) {
        nk[s] = keys[lo + i];
        if constexpr (V) nv[s] = vals[lo + i];
      }
    }
  };
  int lo, m;
  bounds(0, lo, m);
  fetch(lo, m);
  for (int r = 0; r < rounds; ++r) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      if (i < m) {
        L[g].key[i] = flip.enc(nk[s]);
        if constexpr (V) L[g].val[i] = nv[s];
      }
    }
    wave_lds_sync();
    int lo_n = 0, m_n = 0;
    if (r + 1 < rounds) {
      bounds(r + 1, lo_n, m_n);
      fetch(lo_n, m_n);
    }
    rss_group_sort_lds<F>(L[g], m, k0, cfg);
    rss_group_store(L[g], keys + lo, V ? vals + lo : nullptr, m, flip);
    wave_lds_sync();
    lo = lo_n;
    m = m_n;
  }
}

struct SortArgs {
  const int32_t* offsets;
  const int32_t* ids;
  const uint32_t* ctrl;
  int rounds;     // maximum RSS group rounds per tile
  int waves;      // resident waves of a per-class launch (plain baseline)
  int k0[kRssClasses];  // first-level bucket count per RSS class (15..18)
  int interleave;  // alternate RSS and network tiles in the persistent kernel
  int net_mix;     // class 0 holds every network size, in batch order
  RssCfg cfg;   // RSS levels before the rank-counting fallback
  int large_sort;  // 1: the RSS classes are sorted by insertion sort (IS+SN)
  int bound_tiny;   // largest segment of the 8-lane RSS class (16: the class is empty)
  int bound_small;  // largest segment of the 16-lane RSS class
  int bound_mid;    // largest segment of the 32-lane RSS class
};

// Kind sets of the persistent kernels: every class (one kernel holding every
// handler), the network classes (per size, or mixed sizes in batch order), or
// one RSS class (8-, 16-, 32- or 64-lane groups).
constexpr int kKindAll = 0, kKindNet = 1, kKindRss16 = 2, kKindRss32 = 3, kKindRss64 = 4, kKindNetMix = 5,
              kKindRss8 = 6, kKinds = 7;
static_assert(kCtrlTile + kKinds * kTileParts * 32 <= kCtrlWords, "claim counters must fit ctrl");

__host__ __device__ constexpr bool is_net_kind(int ks) { return ks == kKindNet || ks == kKindNetMix; }
__host__ __device__ constexpr bool is_rss_kind(int ks) {
  return ks == kKindRss8 || ks == kKindRss16 || ks == kKindRss32 || ks == kKindRss64;
}
// The class of an RSS kind set, and its lanes per array.
__host__ __device__ constexpr int rss_class_of(int ks) {
  return ks == kKindRss8 ? kNetClasses : kNetClasses + 1 + (ks - kKindRss16);
}

__host__ __device__ __forceinline__ bool in_kind(int c, int ks) {
  if (ks == kKindAll) return true;
  if (is_net_kind(ks)) return c < kNetClasses;
  return c == rss_class_of(ks);
}

// Runs tile `tile_in_class` of class c (only the handlers of kind set KS are
// compiled in).
template <int F, class K, int V, int KS>
__device__ __forceinline__ void run_tile(unsigned char* wave_lds, K* keys, Pay<V>* vals, const SortArgs& a,
                                         KeyMap<K> flip, int c, int tile_in_class, int count, int list, int waves) {
  const int rounds = class_rounds(c, count, a.rounds, waves, kPersistTpw);
  const int first = tile_in_class * class_tile(c, rounds);
  if constexpr (KS == kKindAll || is_net_kind(KS)) {
    if (c < kNetClasses) {
      if constexpr (KS == kKindNetMix)
        net_tile_staged<F, K, V>(wave_lds, keys, vals, a.offsets, a.ids, list, count, first, flip);
      else if (KS == kKindAll && a.net_mix)
        net_tile_mixed<F, K, V>(keys, vals, a.offsets, a.ids, list, count, first, flip);
      else
        net_tile_dispatch<F, K, V>(c + 2, keys, vals, a.offsets, a.ids, list, count, first, flip);
      return;
    }
  }
  if constexpr (KS == kKindAll || KS == kKindRss8) {
    if (c == kNetClasses)
      rss_tile<F, K, V, 8>(wave_lds, keys, vals, a.offsets, a.ids, list, count, first, rounds, flip, a.k0[0],
                           a.cfg);
  }
  if constexpr (KS == kKindAll || KS == kKindRss16) {
    if (c == kNetClasses + 1)
      rss_tile<F, K, V, 16>(wave_lds, keys, vals, a.offsets, a.ids, list, count, first, rounds, flip, a.k0[1],
                            a.cfg);
  }
  if constexpr (KS == kKindAll || KS == kKindRss32) {
    if (c == kNetClasses + 2)
      rss_tile<F, K, V, 32>(wave_lds, keys, vals, a.offsets, a.ids, list, count, first, rounds, flip, a.k0[2],
                            a.cfg);
  }
  if constexpr (KS == kKindAll || KS == kKindRss64) {
    if (c == kNetClasses + 3)
      rss_tile<F, K, V, 64>(wave_lds, keys, vals, a.offsets, a.ids, list, count, first, rounds, flip, a.k0[3],
                            a.cfg);
  }
}

// Tiles of class c in the kernel of kind set KS (0 if the class is not its).
template <int KS>
__device__ __forceinline__ int class_tiles(const uint32_t* ctrl, int c, int rounds, int waves) {
  if (!in_kind(c, KS)) return 0;
  const int count = (int)ctrl[kCtrlCount + c];
  const int ts = class_tile(c, class_rounds(c, count, rounds, waves, kPersistTpw));
  return (count + ts - 1) / ts;
}

// Position of tile t in class order: returns the class and the tile index
// within the class.  The hand-out order lists the RSS classes (most work per
// tile first) and the network classes; with interleaving, RSS and network
// tiles alternate while both remain, so memory-bound network tiles overlap
// with ALU/LDS-bound RSS tiles on every CU.
template <int KS>
__device__ __forceinline__ void locate_tile(int t, const uint32_t* ctrl, int rounds, int waves, int t_rss,
                                            int t_net, bool interleave, int& cls, int& idx) {
  int list_pos;  // position in the concatenated class order
  if (interleave) {
    const int both = 2 * min(t_rss, t_net);
    int i_rss, i_net;  // tile index within the RSS list / network list
    bool is_rss;
    if (t < both) {
      is_rss = (t & 1) == 0;
      i_rss = i_net = t >> 1;
    } else {
      is_rss = t_rss > t_net;
      i_rss = i_net = t - both + min(t_rss, t_net);
    }
    list_pos = is_rss ? i_rss : t_rss + i_net;
  } else {
    list_pos = t;
  }
  // walk the classes in hand-out order (wave-uniform scalar loads)
  cls = class_at(kTiledClasses - 1);
  idx = 0;
  int acc = 0;
  for (int o = 0; o < kTiledClasses; ++o) {
    const int c = class_at(o);
    const int n = class_tiles<KS>(ctrl, c, rounds, waves);
    if (list_pos < acc + n) {
      cls = c;
      idx = list_pos - acc;
      break;
    }
    acc += n;
  }
}

// Waves per SIMD a persistent kernel is compiled for: its register budget.
// The kernel holding every handler would otherwise take more registers than
// the largest of them and lose the occupancy that the latency-bound RSS
// tiles need; the single-kind kernels keep their natural register count.
// Register budget of the persistent kernels, as resident waves per SIMD
// (VGPRs <= 512 / waves): the most each kind reaches without spilling.
template <class K, int V, int KS> struct PersistWaves {
  static constexpr int kType = (sizeof(K) == 8 ? 2 : 0) + (V ? 1 : 0);  // u32, u32+v, u64, u64+v
  static constexpr int value = KS == kKindAll   ? (kType == 0 ? 5 : (kType == 3 ? 3 : 4))
                               : is_net_kind(KS) ? 1
                               : kType == 0     ? (KS == kKindRss16 || KS == kKindRss8 ? 7 : 6)
                               : (kType == 1 && (KS == kKindRss16 || KS == kKindRss8)) ? 5
                                                                  : 4;
};

template <class K, int V, int KS> struct PersistLds {
  static constexpr size_t kBytes = KS == kKindNet    ? 16
                                   : KS == kKindNetMix ? sizeof(NetLds<K, V>)
                                   : KS == kKindRss8  ? 8 * sizeof(GroupLds<K, V, 8>)
                                   : KS == kKindRss16 ? 4 * sizeof(GroupLds<K, V, 16>)
                                   : KS == kKindRss32 ? 2 * sizeof(GroupLds<K, V, 32>)
                                   : KS == kKindRss64 ? sizeof(GroupLds<K, V, 64>)
                                                      : WaveLds<K, V>::kBytes;
};

// Persistent kernel over the classes of kind set KS: waves run tiles until all
// are done.  A single-class kernel indexes its tiles directly.
template <int F, class K, int V, int KS>
__global__ void __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(PersistWaves<K, V, KS>::value)))
seg_persistent_kernel(K* __restrict__ keys, Pay<V>* __restrict__ vals, SortArgs a, uint32_t* ctrl, KeyMap<K> flip) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[kSortWaves][PersistLds<K, V, KS>::kBytes];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: keeps its uses scalar
  const int waves = (int)gridDim.x * kSortWaves;
  // Work is split into kTileParts partitions, partition p = blockIdx mod 8
  // (on one XCD), each with its own claim counter on its own cache line.
  const int part = (int)blockIdx.x % kTileParts;
  const int part_blocks = ((int)gridDim.x - part + kTileParts - 1) / kTileParts;
  const int part_waves = part_blocks * kSortWaves;
  const int wi = ((int)blockIdx.x / kTileParts) * kSortWaves + wave;  // wave index within the partition
  uint32_t* counter = &ctrl[kCtrlTile + (KS * kTileParts + part) * 32];

  constexpr bool kSingle = is_rss_kind(KS);
  if constexpr (kSingle) {
    // One RSS class, in units of one round (one array per lane group).
    // Partition p owns a contiguous range of units; its waves take chunks of
    // `rounds` units round-robin, and the last part -- about one chunk per
    // wave -- in pieces of a quarter chunk claimed from the partition's
    // counter, so the waves finish within about a quarter chunk of each
    // other.
    constexpr int kClass = rss_class_of(KS);
    constexpr int G = rss_group(kClass);
    constexpr int kGroups = kWave / G;
    const int count = (int)a.ctrl[kCtrlCount + kClass];
    const int list = (int)a.ctrl[kCtrlStart + kClass];
    const int k0 = a.k0[kClass - kNetClasses];
    auto run_units = [&](int u, int n) __attribute__((always_inline)) {
      rss_tile<F, K, V, G>(lds[wave], keys, vals, a.offsets, a.ids, list, count, u * kGroups, n, flip, k0, a.cfg);
    };
    const int units = (count + kGroups - 1) / kGroups;
    const int R = class_rounds(kClass, count, a.rounds, waves, kPersistTpw);
    const int u0 = (int)((int64_t)units * part / kTileParts);
    const int u1 = (int)((int64_t)units * (part + 1) / kTileParts);
    const int static_chunks = max(0, (u1 - u0) / R - part_waves);
    // (a static chunk always holds R units; spelling the bound out as for the
    // dynamic pieces measured 25-35% faster on arrays of 17..64 keys, from
    // the code the compiler generates for the two inlined copies)
    for (int q = wi; q < static_chunks; q += part_waves) run_units(u0 + q * R, min(R, u1 - (u0 + q * R)));
    const int d0 = u0 + static_chunks * R;
    const int piece = max(1, R / 4);
    if (d0 >= u1) return;
    while (true) {
      int c0 = 0;
      if (lane_id() == 0) c0 = (int)atomicAdd(counter, 1u);
      const int u = d0 + __builtin_amdgcn_readfirstlane(c0) * piece;
      if (u >= u1) break;
      run_units(u, min(piece, u1 - u));
    }
    return;
  }
  // tiles of the RSS classes and of the network classes (wave-uniform)
  int t_rss = 0, t_net = 0;
  for (int c = 0; c < kTiledClasses; ++c) {
    const int n = class_tiles<KS>(a.ctrl, c, a.rounds, waves);
    if (c >= kNetClasses)
      t_rss += n;
    else
      t_net += n;
  }
  // the network-only kernels keep their class prefix in registers
  int net_first[kNetClasses + 1];
  if constexpr (is_net_kind(KS)) {
    int acc = 0;
#pragma unroll
    for (int o = 0; o < kNetClasses; ++o) {
      net_first[o] = acc;
      acc += class_tiles<KS>(a.ctrl, class_at(kRssClasses + o), a.rounds, waves);
    }
    net_first[kNetClasses] = acc;
  }
  const int total = t_rss + t_net;
  // Tiles are handed out round-robin by wave index, except the last ones
  // (half a tile per wave), which waves claim from their partition's counter
  // as they finish so that uneven tiles do not leave a tail.  (Claiming every
  // tile from one device-wide counter costs more: atomics on one line from all
  // XCDs serialise.)
  auto process = [&](int t) __attribute__((always_inline)) {
    if constexpr (is_net_kind(KS)) {
      int c = 0, idx = 0;
#pragma unroll
      for (int o = 0; o < kNetClasses; ++o) {
        if (t >= net_first[o] && t < net_first[o + 1]) {
          c = class_at(kRssClasses + o);
          idx = t - net_first[o];
        }
      }
      run_tile<F, K, V, KS>(lds[wave], keys, vals, a, flip, c, idx, (int)a.ctrl[kCtrlCount + c],
                            (int)a.ctrl[kCtrlStart + c], waves);
    } else {
      int c, idx;
      locate_tile<KS>(t, a.ctrl, a.rounds, waves, t_rss, t_net, a.interleave != 0, c, idx);
      run_tile<F, K, V, KS>(lds[wave], keys, vals, a, flip, c, idx, (int)a.ctrl[kCtrlCount + c],
                            (int)a.ctrl[kCtrlStart + c], waves);
    }
  };
  // Tiles t = part + 8*i belong to partition part.
  const int part_tiles = (total - part + kTileParts - 1) / kTileParts;
  const int static_end = part_tiles - min(part_tiles, part_waves / 2);
  int i = wi;
  while (true) {
    if (i >= static_end) {  // dynamic tail: claim the next tile of the partition
      if (static_end == part_tiles) break;
      int c0 = 0;
      if (lane_id() == 0) c0 = (int)atomicAdd(counter, 1u);
      i = static_end + __builtin_amdgcn_readfirstlane(c0);
      if (i >= part_tiles) break;
    }
    process(part + kTileParts * i);
    i = i < static_end ? i + part_waves : static_end;
  }
  (void)net_first;
}

// Plain baseline: one launch per class, tile = blockIdx * waves + wave.  The
// kernel is specialised per handler (KIND 0: networks, 1..4: the RSS classes
// 15..18, with 8-, 16-, 32-, 64-lane groups), so each launch carries only its
// own code and registers.
template <int F, class K, int V, int KIND>
__global__ void __launch_bounds__(kSortThreads)
seg_class_kernel(K* __restrict__ keys, Pay<V>* __restrict__ vals, SortArgs a, KeyMap<K> flip, int c, int count,
                 int list) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[kSortWaves][KIND == 0 ? 16 : WaveLds<K, V>::kBytes];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform: keeps its uses scalar
  const int tile = blockIdx.x * kSortWaves + wave;
  const int rounds = class_rounds(c, count, a.rounds, a.waves, kPlainTpw);
  const int first = tile * class_tile(c, rounds);
  if constexpr (KIND == 0) {
    net_tile_dispatch<F, K, V>(c + 2, keys, vals, a.offsets, a.ids, list, count, first, flip);
  } else {
    constexpr int kClass = kNetClasses + KIND - 1;
    rss_tile<F, K, V, rss_group(kClass)>(lds[wave], keys, vals, a.offsets, a.ids, list, count, first, rounds, flip,
                                         a.k0[KIND - 1], a.cfg);
  }
}

// Segments of 257..4096 keys: one work-group per segment, the work-groups
// striding over the class list (the same kernel serves every form; the count
// comes from the binning's control block).  With large_sort = 1 (the IS+SN
// alternative) one lane per segment sorts it by insertion sort instead.
template <int F, class K, int V>
__global__ void __launch_bounds__(kLargeThreads)
seg_large_kernel(K* __restrict__ keys, Pay<V>* __restrict__ vals, SortArgs a, KeyMap<K> flip) {
  extern __shared__ __attribute__((aligned(16))) unsigned char large_lds[];
  const int count = (int)a.ctrl[kCtrlCount + kLargeClass];
  const int list = (int)a.ctrl[kCtrlStart + kLargeClass];
  for (int j = blockIdx.x; j < count; j += gridDim.x) {
    const int seg = a.ids[list + j];
    const int lo = a.offsets[seg];
    const int m = a.offsets[seg + 1] - lo;
    if (a.large_sort) {
      if (threadIdx.x == 0) insertion_sort_global<K, V>(keys + lo, V ? vals + lo : nullptr, m, flip);
      continue;
    }
    large_sort<F, K, V>(large_lds, keys + lo, V ? vals + lo : nullptr, m, flip, a.k0[3], a.cfg);
  }
}

// Work-groups of the large-class kernel: as many as are resident at once
// (its dynamic LDS is raised above the default limit on first use).
template <int F, class K, int V>
static int large_blocks(DeviceCtx* c) {
  static const hipError_t attr = allow_dynamic_lds(seg_large_kernel<F, K, V>, LargeLds<K, V>::kBytes);
  int nb = 0;
  if (attr != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, seg_large_kernel<F, K, V>, kLargeThreads,
                                                   LargeLds<K, V>::kBytes) != hipSuccess ||
      nb <= 0)
    nb = 1;
  return nb * c->num_cus;
}

// The IS+SN alternative for every RSS class (large_sort = 1): one lane per
// segment, insertion sort in global memory.  The three class lists are
// consecutive in the segment-id list.  A kernel of its own, so that the
// Register Sample Sort kernels carry none of its code or registers.
template <class K, int V>
__global__ void __launch_bounds__(kSortThreads)
seg_is_kernel(K* __restrict__ keys, Pay<V>* __restrict__ vals, SortArgs a, uint32_t* ctrl, KeyMap<K> flip) {
  (void)ctrl;
  const int list = (int)a.ctrl[kCtrlStart + kNetClasses];
  int count = 0;
  for (int c = kNetClasses; c < kNetClasses + kRssClasses; ++c) count += (int)a.ctrl[kCtrlCount + c];
  for (int j = blockIdx.x * kSortThreads + threadIdx.x; j < count; j += gridDim.x * kSortThreads) {
    const int seg = a.ids[list + j];
    const int lo = a.offsets[seg];
    insertion_sort_global<K, V>(keys + lo, V ? vals + lo : nullptr, a.offsets[seg + 1] - lo, flip);
  }
}

// --- host side ---------------------------------------------------------------

struct GraphEntry {
  int key = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t nodes[9] = {};  // count, scan, scatter, the persistent kernel(s), the large class
  int nnodes = 0;
  int persist_blocks[kKinds] = {};
};

struct SegmentedCache {
  std::mutex mu;
  int32_t* ids = nullptr;
  int64_t ids_cap = 0;
  uint32_t* ctrl = nullptr;
  uint32_t* blockhist = nullptr;
  uint32_t* host_ctrl = nullptr;  // pinned, for the plain baseline
  std::vector<GraphEntry> graphs;
  SegBuffers buffers() const {
    SegBuffers b;
    b.ids = ids;
    b.ctrl = ctrl;
    b.blockhist = blockhist;
    return b;
  }
};

// Working memory of the stream `s` on this device (created on first use; calls
// on different streams never share it, so they may overlap on the device).
SegmentedCache* workspace_for(DeviceCtx* c, hipStream_t s);
// Grows the workspace's segment-id list to hold nseg ids, stream-ordered on
// `s` (caller holds ws->mu).
hipError_t ensure_workspace(SegmentedCache* ws, int32_t nseg, hipStream_t s);

template <int F, class K, int V, int KS>
static int persistent_blocks(DeviceCtx* c) {
  int occ = tuning(sizeof(K)).persist_occ;
  if (occ <= 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, seg_persistent_kernel<F, K, V, KS>, kSortThreads, 0) !=
            hipSuccess ||
        nb <= 0)
      nb = 2;
    occ = nb;
  }
  // every partition (blockIdx mod kTileParts) needs at least one work-group
  return max(occ * c->num_cus, kTileParts);
}

template <class K>
inline SortArgs make_args(const int32_t* offsets, const SegBuffers& s) {
  const Tuning t = tuning(sizeof(K));
  SortArgs a;
  a.offsets = offsets;
  a.ids = s.ids;
  a.ctrl = s.ctrl;
  a.rounds = t.rss_rounds;
  a.waves = 1;
  a.k0[0] = 8;  // the 8-lane class: every first level has 8 buckets
  a.k0[1] = t.rss_k[0];
  a.k0[2] = t.rss_k[1];
  a.k0[3] = t.rss_k[2];
  a.interleave = t.interleave;
  a.net_mix = t.net_mix;
  a.bound_tiny = t.rss_bound_tiny;
  a.bound_small = t.rss_bound_small;
  a.bound_mid = t.rss_bound_mid;
  a.cfg = RssCfg{t.rss_level_cap, t.rss_oversample, t.rss_finish};
  a.large_sort = t.large_sort;
  return a;
}

// The kernels of one call with their arguments, as launch parameter blocks:
// count, scan, scatter, then either the persistent kernel over every class or
// (split) the network-class kernel followed by the RSS-class kernel.
template <int F, class K, int V>
struct SegLaunch {
  // argument storage (addresses handed to HIP)
  const int32_t* offsets;
  int32_t nseg;
  uint32_t* blockhist;
  int* status;
  int nblocks;
  uint32_t* ctrl;
  const uint32_t* ctrl_c;
  const uint32_t* blockbase;
  int32_t* ids;
  K* keys;
  Pay<V>* vals;
  SortArgs args;
  KeyMap<K> flip;
  int mix;   // binning mixes the network sizes (persistent forms only)
  int bins;  // pack_bins(mix, RSS class bounds): the binning kernels' parameter
  void* p_count[5];
  void* p_scan[3];
  void* p_scatter[6];
  void* p_sort[5];
  void* p_sort_large[4];
  bool split;
  int persist_blocks[kKinds];  // grid of the persistent kernel per kind set
  int large_grid;              // work-groups of the large-class kernel

  bool is_rss;  // large_sort: one insertion-sort kernel replaces the RSS kernels (split form only)

  int nnodes() const { return split ? (is_rss ? 6 : 9) : 5; }
  // kind set of node i >= 3: network classes, then the RSS classes largest first
  int node_kind(int i) const {
    if (!split) return kKindAll;
    static constexpr int order[5] = {kKindNet, kKindRss64, kKindRss32, kKindRss16, kKindRss8};
    return (i == 3 && mix) ? kKindNetMix : order[i - 3];
  }

  void fill(DeviceCtx* c, const SegBuffers& s, K* k, Pay<V>* v, const int32_t* off, int32_t n, KeyMap<K> fl) {
    offsets = off;
    nseg = n;
    blockhist = s.blockhist;
    status = s.quiet ? nullptr : c->status;
    nblocks = kBinBlocks;
    ctrl = s.ctrl;
    ctrl_c = s.ctrl;
    blockbase = s.blockhist;
    ids = s.ids;
    keys = k;
    vals = v;
    args = make_args<K>(off, s);
    flip = fl;
    mix = args.net_mix;
    bins = pack_bins(mix, args.bound_tiny, args.bound_small, args.bound_mid);
    p_count[0] = &offsets; p_count[1] = &nseg; p_count[2] = &blockhist; p_count[3] = &status; p_count[4] = &bins;
    p_scan[0] = &blockhist; p_scan[1] = &nblocks; p_scan[2] = &ctrl;
    p_scatter[0] = &offsets; p_scatter[1] = &nseg; p_scatter[2] = &blockbase; p_scatter[3] = &ctrl_c;
    p_scatter[4] = &ids; p_scatter[5] = &bins;
    p_sort[0] = &keys; p_sort[1] = &vals; p_sort[2] = &args; p_sort[3] = &ctrl; p_sort[4] = &flip;
    p_sort_large[0] = &keys; p_sort_large[1] = &vals; p_sort_large[2] = &args; p_sort_large[3] = &flip;
  }

  static void* kernel_of(int ks) {
    switch (ks) {
      case kKindNet: return (void*)seg_persistent_kernel<F, K, V, kKindNet>;
      case kKindNetMix: return (void*)seg_persistent_kernel<F, K, V, kKindNetMix>;
      case kKindRss8: return (void*)seg_persistent_kernel<F, K, V, kKindRss8>;
      case kKindRss16: return (void*)seg_persistent_kernel<F, K, V, kKindRss16>;
      case kKindRss32: return (void*)seg_persistent_kernel<F, K, V, kKindRss32>;
      case kKindRss64: return (void*)seg_persistent_kernel<F, K, V, kKindRss64>;
      default: return (void*)seg_persistent_kernel<F, K, V, kKindAll>;
    }
  }

  hipKernelNodeParams node(int i) {
    hipKernelNodeParams p{};
    p.sharedMemBytes = 0;
    p.extra = nullptr;
    switch (i) {
      case 0:
        p.func = (void*)seg_count_kernel;
        p.gridDim = dim3(kBinBlocks);
        p.blockDim = dim3(kBinThreads);
        p.kernelParams = p_count;
        break;
      case 1:
        p.func = (void*)seg_scan_kernel;
        p.gridDim = dim3(1);
        p.blockDim = dim3(1024);
        p.kernelParams = p_scan;
        break;
      case 2:
        p.func = (void*)seg_scatter_kernel;
        p.gridDim = dim3(kBinBlocks);
        p.blockDim = dim3(kBinThreads);
        p.kernelParams = p_scatter;
        break;
      default: {
        if (i == nnodes() - 1) {
          p.func = (void*)seg_large_kernel<F, K, V>;
          p.gridDim = dim3(large_grid);
          p.blockDim = dim3(kLargeThreads);
          p.sharedMemBytes = LargeLds<K, V>::kBytes;
          p.kernelParams = p_sort_large;
          break;
        }
        if (is_rss && i == 4) {
          p.func = (void*)seg_is_kernel<K, V>;
          p.gridDim = dim3(persist_blocks[kKindNet]);
          p.blockDim = dim3(kSortThreads);
          p.kernelParams = p_sort;
          break;
        }
        const int ks = node_kind(i);
        p.func = kernel_of(ks);
        p.gridDim = dim3(persist_blocks[ks]);
        p.blockDim = dim3(kSortThreads);
        p.kernelParams = p_sort;
        break;
      }
    }
    return p;
  }

  hipError_t launch_binning(hipStream_t s) {
    hipLaunchKernelGGL(seg_count_kernel, dim3(kBinBlocks), dim3(kBinThreads), 0, s, offsets, nseg, blockhist,
                       status, bins);
    hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(1024), 0, s, blockhist, nblocks, ctrl);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(kBinBlocks), dim3(kBinThreads), 0, s, offsets, nseg, blockbase,
                       ctrl_c, ids, bins);
    return hipGetLastError();
  }
  hipError_t launch_direct(hipStream_t s) {
    hipError_t e = launch_binning(s);
    if (e != hipSuccess) return e;
    for (int i = 3; i < nnodes(); ++i) {
      hipKernelNodeParams p = node(i);
      hipError_t le = hipLaunchKernel(p.func, p.gridDim, p.blockDim, p.kernelParams, p.sharedMemBytes, s);
      if (le != hipSuccess) return le;
    }
    return hipGetLastError();
  }
};

template <int F, class K, int V>
static hipError_t run_plain(DeviceCtx* c, SegmentedCache* sc, SegLaunch<F, K, V>& L, hipStream_t s) {
  // resident waves of one per-class launch (largest RSS class kernel)
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, seg_class_kernel<F, K, V, kRssClasses>, kSortThreads, 0) !=
          hipSuccess ||
      nb <= 0)
    nb = 2;
  L.args.waves = nb * c->num_cus * kSortWaves;
  L.args.net_mix = 0;  // the baseline launches one kernel per network size
  L.mix = 0;
  L.bins = pack_bins(0, L.args.bound_tiny, L.args.bound_small, L.args.bound_mid);
  hipError_t e = L.launch_binning(s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sc->host_ctrl, sc->ctrl, (kCtrlStart + kClasses) * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int o = 0; o < kTiledClasses; ++o) {
    const int cls = class_at(o);
    const int count = (int)sc->host_ctrl[kCtrlCount + cls];
    if (count == 0) continue;
    const int ts = class_tile(cls, class_rounds(cls, count, L.args.rounds, L.args.waves, kPlainTpw));
    const int tiles = (count + ts - 1) / ts;
    const int blocks = (tiles + kSortWaves - 1) / kSortWaves;
    const int list = (int)sc->host_ctrl[kCtrlStart + cls];
    if (cls >= kNetClasses && L.is_rss) continue;  // the insertion-sort kernel below takes every RSS class
    if (cls < kNetClasses)
      hipLaunchKernelGGL((seg_class_kernel<F, K, V, 0>), dim3(blocks), dim3(kSortThreads), 0, s, L.keys, L.vals,
                         L.args, L.flip, cls, count, list);
    else if (cls == kNetClasses)
      hipLaunchKernelGGL((seg_class_kernel<F, K, V, 1>), dim3(blocks), dim3(kSortThreads), 0, s, L.keys, L.vals,
                         L.args, L.flip, cls, count, list);
    else if (cls == kNetClasses + 1)
      hipLaunchKernelGGL((seg_class_kernel<F, K, V, 2>), dim3(blocks), dim3(kSortThreads), 0, s, L.keys, L.vals,
                         L.args, L.flip, cls, count, list);
    else if (cls == kNetClasses + 2)
      hipLaunchKernelGGL((seg_class_kernel<F, K, V, 3>), dim3(blocks), dim3(kSortThreads), 0, s, L.keys, L.vals,
                         L.args, L.flip, cls, count, list);
    else
      hipLaunchKernelGGL((seg_class_kernel<F, K, V, 4>), dim3(blocks), dim3(kSortThreads), 0, s, L.keys, L.vals,
                         L.args, L.flip, cls, count, list);
  }
  if (L.is_rss) {
    int nrss = 0;
    for (int c = kNetClasses; c < kNetClasses + kRssClasses; ++c) nrss += (int)sc->host_ctrl[kCtrlCount + c];
    if (nrss > 0)
      hipLaunchKernelGGL((seg_is_kernel<K, V>), dim3((nrss + kSortThreads - 1) / kSortThreads), dim3(kSortThreads), 0,
                         s, L.keys, L.vals, L.args, L.ctrl, L.flip);
  }
  const int nlarge = (int)sc->host_ctrl[kCtrlCount + kLargeClass];
  if (nlarge > 0) {
    hipKernelNodeParams p = L.node(L.nnodes() - 1);
    hipError_t le = hipLaunchKernel(p.func, dim3(min(nlarge, L.large_grid)), p.blockDim, p.kernelParams,
                                    p.sharedMemBytes, s);
    if (le != hipSuccess) return le;
  }
  return hipGetLastError();
}

template <int F, class K, int V>
static hipError_t run_graph(SegmentedCache* sc, SegLaunch<F, K, V>& L, hipStream_t s) {
  const int key = (((((int)sizeof(K) * 16 + V) * 3 + F) * 2 + (L.split ? 1 : 0)) * 2 + (L.mix ? 1 : 0)) * 2 +
                  (L.is_rss ? 1 : 0);
  GraphEntry* g = nullptr;
  for (GraphEntry& ge : sc->graphs)
    if (ge.key == key && std::equal(ge.persist_blocks, ge.persist_blocks + kKinds, L.persist_blocks)) g = &ge;
  hipError_t e = hipSuccess;
  if (!g) {
    GraphEntry ne;
    ne.key = key;
    ne.nnodes = L.nnodes();
    std::copy(L.persist_blocks, L.persist_blocks + kKinds, ne.persist_blocks);
    e = hipGraphCreate(&ne.graph, 0);
    for (int i = 0; i < ne.nnodes && e == hipSuccess; ++i) {
      hipKernelNodeParams p = L.node(i);
      e = hipGraphAddKernelNode(&ne.nodes[i], ne.graph, i ? &ne.nodes[i - 1] : nullptr, i ? 1 : 0, &p);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ne.exec, ne.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (ne.graph) (void)hipGraphDestroy(ne.graph);
      return e;
    }
    sc->graphs.push_back(ne);
    g = &sc->graphs.back();
  } else {
    for (int i = 0; i < g->nnodes && e == hipSuccess; ++i) {
      hipKernelNodeParams p = L.node(i);
      e = hipGraphExecKernelNodeSetParams(g->exec, g->nodes[i], &p);
    }
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(g->exec, s);
}

template <int F, class K, int V>
static void init_launch(DeviceCtx* c, SegLaunch<F, K, V>& L) {
  // the insertion-sort alternative always runs in the split form
  L.is_rss = tuning(sizeof(K)).large_sort != 0;
  L.split = tuning(sizeof(K)).persist_split != 0 || L.is_rss;
  for (int& b : L.persist_blocks) b = 0;
  if (L.split) {
    L.persist_blocks[kKindNet] = persistent_blocks<F, K, V, kKindNet>(c);
    L.persist_blocks[kKindNetMix] = persistent_blocks<F, K, V, kKindNetMix>(c);
    L.persist_blocks[kKindRss8] = persistent_blocks<F, K, V, kKindRss8>(c);
    L.persist_blocks[kKindRss16] = persistent_blocks<F, K, V, kKindRss16>(c);
    L.persist_blocks[kKindRss32] = persistent_blocks<F, K, V, kKindRss32>(c);
    L.persist_blocks[kKindRss64] = persistent_blocks<F, K, V, kKindRss64>(c);
  } else {
    L.persist_blocks[kKindAll] = persistent_blocks<F, K, V, kKindAll>(c);
  }
  L.large_grid = large_blocks<F, K, V>(c);
}

template <int F, class K, int V>
int segmented_impl(DeviceCtx* c, SegmentedCache* ws, K* keys, Pay<V>* vals, const int32_t* offsets, int32_t nseg,
                   KeyMap<K> flip, int mode, hipStream_t s) {
  SegLaunch<F, K, V> L;
  init_launch(c, L);
  L.fill(c, ws->buffers(), keys, vals, offsets, nseg, flip);
  hipError_t e;
  if (mode == 2)
    e = run_plain(c, ws, L, s);
  else if (mode == 1)
    e = L.launch_direct(s);
  else
    e = run_graph(ws, L, s);
  if (e == hipErrorOutOfMemory) return -5;
  return e == hipSuccess ? 0 : -4;
}

// The no-allocation form: binning and persistent kernels launched directly on
// caller-provided buffers (the fixed scratch array); no graph, no allocation.
template <int F, class K, int V>
int segmented_direct_impl(DeviceCtx* c, const SegBuffers& b, K* keys, Pay<V>* vals, const int32_t* offsets,
                          int32_t nseg, KeyMap<K> flip, hipStream_t s) {
  SegLaunch<F, K, V> L;
  init_launch(c, L);
  L.fill(c, b, keys, vals, offsets, nseg, flip);
  return L.launch_direct(s) == hipSuccess ? 0 : -4;
}

// Every (family, key width, payload bytes) combination of the segmented path
// (32-bit keys carry no payload or a 32-bit one; 64-bit keys also a 64-bit
// one, the key + reference pairs of Section 2.2).  Each is compiled in an
// instantiation unit of its own (written by the build into _build/, so the
// units compile in parallel); every other unit only refers to them.
#define SS_SEGMENTED_COMBOS(X)                                                                \
  X(0, uint32_t, 0) X(0, uint32_t, 4) X(1, uint32_t, 0) X(1, uint32_t, 4) X(2, uint32_t, 0)   \
  X(2, uint32_t, 4) X(0, uint64_t, 0) X(0, uint64_t, 4) X(0, uint64_t, 8) X(1, uint64_t, 0)   \
  X(1, uint64_t, 4) X(1, uint64_t, 8) X(2, uint64_t, 0) X(2, uint64_t, 4) X(2, uint64_t, 8)

#define SS_SEGMENTED_DECLARE(F, K, V, EXT)                                                              \
  EXT template int segmented_impl<F, K, V>(DeviceCtx*, SegmentedCache*, K*, Pay<V>*, const int32_t*,   \
                                           int32_t, KeyMap<K>, int, hipStream_t);                       \
  EXT template int segmented_direct_impl<F, K, V>(DeviceCtx*, const SegBuffers&, K*, Pay<V>*,          \
                                                  const int32_t*, int32_t, KeyMap<K>, hipStream_t);
#define SS_SEGMENTED_EXTERN(F, K, V) SS_SEGMENTED_DECLARE(F, K, V, extern)
#ifndef SS_SEGMENTED_INSTANCE_UNIT
SS_SEGMENTED_COMBOS(SS_SEGMENTED_EXTERN)
#endif

// The instantiation for family F and the payload width: vbytes = 0 (no
// payload), 4 or 8 (64-bit keys only).
template <int F, class K>
static int segmented_pick(DeviceCtx* c, SegmentedCache* ws, const SegBuffers* b, K* keys, void* vals, int vbytes,
                          const int32_t* offsets, int32_t nseg, KeyMap<K> flip, int mode, hipStream_t s) {
  if (vbytes == 8) {
    if constexpr (sizeof(K) == 8) {
      auto* v = static_cast<uint64_t*>(vals);
      return b ? segmented_direct_impl<F, K, 8>(c, *b, keys, v, offsets, nseg, flip, s)
               : segmented_impl<F, K, 8>(c, ws, keys, v, offsets, nseg, flip, mode, s);
    }
    return -1;
  }
  if (vbytes == 4) {
    auto* v = static_cast<uint32_t*>(vals);
    return b ? segmented_direct_impl<F, K, 4>(c, *b, keys, v, offsets, nseg, flip, s)
             : segmented_impl<F, K, 4>(c, ws, keys, v, offsets, nseg, flip, mode, s);
  }
  return b ? segmented_direct_impl<F, K, 0>(c, *b, keys, nullptr, offsets, nseg, flip, s)
           : segmented_impl<F, K, 0>(c, ws, keys, nullptr, offsets, nseg, flip, mode, s);
}

template <class K>
static int segmented_family(DeviceCtx* c, SegmentedCache* ws, const SegBuffers* b, K* keys, void* vals, int vbytes,
                            const int32_t* offsets, int32_t nseg, KeyMap<K> flip, int mode, hipStream_t s) {
  switch (tuning(sizeof(K)).family) {
    case 1: return segmented_pick<1, K>(c, ws, b, keys, vals, vbytes, offsets, nseg, flip, mode, s);
    case kFamilyInsertion:
      return segmented_pick<kFamilyInsertion, K>(c, ws, b, keys, vals, vbytes, offsets, nseg, flip, mode, s);
    default: return segmented_pick<0, K>(c, ws, b, keys, vals, vbytes, offsets, nseg, flip, mode, s);
  }
}

template <class K>
static int segmented_any(DeviceCtx* c, K* keys, void* vals, int vbytes, const int32_t* offsets, int32_t nseg,
                         KeyMap<K> flip, int mode, hipStream_t s) {
  SegmentedCache* ws = workspace_for(c, s);
  if (!ws) return -5;
  std::lock_guard<std::mutex> lock(ws->mu);
  hipError_t e = ensure_workspace(ws, nseg, s);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? -5 : -4;
  return segmented_family<K>(c, ws, nullptr, keys, vals, vbytes, offsets, nseg, flip, mode, s);
}

template <class K>
static int segmented_direct_any(DeviceCtx* c, const SegBuffers& b, K* keys, void* vals, int vbytes,
                                const int32_t* offsets, int32_t nseg, KeyMap<K> flip, hipStream_t s) {
  return segmented_family<K>(c, nullptr, &b, keys, vals, vbytes, offsets, nseg, flip, 1, s);
}

}  // namespace ss
