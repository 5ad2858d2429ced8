// Register Sample Sort (paper, Section 3) for one array of 17..256 keys,
// executed by a group of G lanes (G = 16, 32 or 64) of a wave.
//
// The array is staged in LDS.  Each level of the recursion handles every
// pending bucket (more than 16 keys) of the array:
//
//   1. sample: one lane per pending bucket picks 16 keys at equidistant
//      positions floor((2t+1)*size/32), t = 0..15, and sorts them with the
//      16-channel network (Section 3: "the same sorting method can be used as
//      for the base case");
//   2. splitters: s_i = S_{a*i} for i = 1..k-1 with k buckets and
//      oversampling a = 16/k (Section 3, basic sample sort);
//   3. classify: bucket j = #{splitters < e}, i.e. s_j < e <= s_{j+1}, found
//      by descending the perfect splitter tree without branches: compare with
//      the root, then keep either the left or the right subtree with selects
//      (the paper's "unconditional copy of the left subtree, conditionally
//      overwritten with the right one"), and append the comparison bit to the
//      bucket index, j = 2j + [e > root];
//   4. scatter: a stable multisplit -- per-slot ballots of the bucket-index
//      bits give each key its rank among equal buckets, per-bucket counts are
//      scanned into offsets -- and the keys are written back in bucket order;
//   5. buckets of 2..16 keys join the finish list, larger ones are pending
//      for the next level (the paper recurses until buckets are at most 16).
//
// Buckets on the finish list are sorted one per lane: the bucket is loaded
// into the channels 0..m-1 of a network of the smallest size covering every
// bucket of the wave, channels m.. are filled with the maximum key, and the
// strict compare-exchange never moves a padding channel (a channel >= m holds
// the maximum, which no real key exceeds), so channels 0..m-1 end sorted.
//
// Termination with duplicate keys (not covered by the paper): if all k-1
// splitters of a bucket are equal to v, the bucket is split three ways,
// {e < v}, {e == v}, {e > v}; the middle part is already in final order.  Every
// other split sends the smallest splitter's key to bucket 0 and the largest
// splitter's key above it, so every child is strictly smaller than its parent.
// After kLevelCap levels any remaining pending bucket is finished by a
// rank-counting sort (each key's final position is the number of keys that
// must precede it), which is always correct.
#pragma once

#include "common.hpp"

namespace ss {

constexpr int kLevelCap = 8;

template <class K, bool V, int G> struct GroupLds {
  static constexpr int kCap = 4 * G;          // keys per array handled by a G-lane group
  static constexpr int kMaxPend = kCap / 17;  // buckets with more than 16 keys
  static constexpr int kMaxFin = kCap / 2;    // buckets with 2..16 keys
  K key[kCap];
  uint32_t val[V ? kCap : 1];
  K sample[kMaxPend][16];
  uint16_t pend_st[2][kMaxPend];
  uint16_t pend_sz[2][kMaxPend];
  uint16_t fin_st[kMaxFin];
  uint16_t fin_sz[kMaxFin];
};

// Orders this wave's LDS accesses: DS instructions of one wave execute in
// order, so only the compiler must be kept from moving accesses across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d));
  return x;
}

// Splitter-tree descent over a sorted subtree sub[0..W-1], W = 2^L - 1.
template <int L, class K> struct TreeDescent {
  __device__ __forceinline__ static int run(K e, const K* sub, int j) {
    constexpr int W = (1 << L) - 1;
    constexpr int H = W / 2;  // size of each child subtree
    const bool b = e > sub[H];
    j = 2 * j + (b ? 1 : 0);
    if constexpr (L > 1) {
      K next[H];
#pragma unroll
      for (int t = 0; t < H; ++t) next[t] = b ? sub[H + 1 + t] : sub[t];
      return TreeDescent<L - 1, K>::run(e, next, j);
    } else {
      return j;
    }
  }
};

// Bucket index of e among the k-1 = 2^LOGK - 1 sorted splitters spl[].
template <int LOGK, class K>
__device__ __forceinline__ int classify(K e, const K* spl) {
  return TreeDescent<LOGK, K>::run(e, spl, 0);
}

// Finish the buckets of the finish list with networks of N channels.
template <int F, int N, class K, bool V, int G>
__device__ __forceinline__ void finish_buckets(GroupLds<K, V, G>& L, bool ok, int st, int sz) {
  K r[N];
  uint32_t v[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool in = ok && j < sz;
    r[j] = in ? L.key[st + j] : KeyTraits<K>::kMax;
    if constexpr (V) v[j] = in ? L.val[st + j] : 0u;
  }
  if constexpr (V)
    net_sort<F, N>(r, v);
  else
    net_sort<F, N>(r);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (ok && j < sz) {
      L.key[st + j] = r[j];
      if constexpr (V) L.val[st + j] = v[j];
    }
  }
}

template <int F, class K, bool V, int G>
__device__ __forceinline__ void finish_dispatch(GroupLds<K, V, G>& L, bool ok, int st, int sz, int nmax) {
  switch (nmax) {
    case 2: finish_buckets<F, 2>(L, ok, st, sz); break;
    case 3: finish_buckets<F, 3>(L, ok, st, sz); break;
    case 4: finish_buckets<F, 4>(L, ok, st, sz); break;
    case 5: finish_buckets<F, 5>(L, ok, st, sz); break;
    case 6: finish_buckets<F, 6>(L, ok, st, sz); break;
    case 7: finish_buckets<F, 7>(L, ok, st, sz); break;
    case 8: finish_buckets<F, 8>(L, ok, st, sz); break;
    case 9: finish_buckets<F, 9>(L, ok, st, sz); break;
    case 10: finish_buckets<F, 10>(L, ok, st, sz); break;
    case 11: finish_buckets<F, 11>(L, ok, st, sz); break;
    case 12: finish_buckets<F, 12>(L, ok, st, sz); break;
    case 13: finish_buckets<F, 13>(L, ok, st, sz); break;
    case 14: finish_buckets<F, 14>(L, ok, st, sz); break;
    case 15: finish_buckets<F, 15>(L, ok, st, sz); break;
    default: finish_buckets<F, 16>(L, ok, st, sz); break;
  }
}

// One level of classification + scatter for the pending buckets, k = 2^LOGK.
template <int LOGK, class K, bool V, int G>
__device__ __forceinline__ void split_level(GroupLds<K, V, G>& L, int cur, int np, int& nf, int& npn) {
  constexpr int k = 1 << LOGK;
  constexpr int a = 16 / k;  // oversampling factor
  const int lane = lane_id();
  const int gl = lane % G;
  const int gbase = lane - gl;
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  const uint64_t below = (1ull << lane) - 1ull;

  for (int p = 0; ballot(p < np) != 0ull; ++p) {
    const bool active = p < np;
    const int st = active ? (int)L.pend_st[cur][p] : 0;
    const int sz = active ? (int)L.pend_sz[cur][p] : 0;
    K spl[k - 1];
#pragma unroll
    for (int i = 0; i < k - 1; ++i) spl[i] = active ? L.sample[p][a * (i + 1) - 1] : K(0);
    const bool degenerate = active && spl[0] == spl[k - 2];
    const int nch = degenerate ? 3 : k;

    K e[4];
    uint32_t v[4];
    int c[4];
    bool ok[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      ok[s] = active && i < sz;
      e[s] = ok[s] ? L.key[st + i] : K(0);
      if constexpr (V) v[s] = ok[s] ? L.val[st + i] : 0u;
      int cc = classify<LOGK>(e[s], spl);
      int cd = e[s] < spl[0] ? 0 : (e[s] == spl[0] ? 1 : 2);
      c[s] = degenerate ? cd : cc;
    }

    // stable multisplit: rank within slot, per-child running counts
    uint32_t cnt = 0;
    uint32_t pre[4];
    uint32_t rank[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint64_t A = ballot(ok[s]) & gmask;
      uint64_t my = A, mq = A;
#pragma unroll
      for (int b = 0; b < LOGK; ++b) {
        const uint64_t B = ballot(ok[s] && ((c[s] >> b) & 1));
        my &= ((c[s] >> b) & 1) ? B : ~B;
        mq &= ((gl >> b) & 1) ? B : ~B;
      }
      rank[s] = (uint32_t)__popcll(my & below);
      pre[s] = cnt;
      cnt += (uint32_t)__popcll(mq);
    }
    // exclusive scan of the child counts over lanes gl < nch of the group
    const uint32_t x = (gl < nch) ? cnt : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      uint32_t y = read_lane(incl, gl >= d ? lane - d : lane);
      if (gl >= d) incl += y;
    }
    const uint32_t off = incl - x;
    int pos[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint32_t base = read_lane(off + pre[s], gbase + (c[s] & 15));
      pos[s] = st + (int)(base + rank[s]);
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (ok[s]) {
        L.key[pos[s]] = e[s];
        if constexpr (V) L.val[pos[s]] = v[s];
      }
    }
    // children of this bucket: lane gl describes child gl
    const bool own = active && gl < nch;
    const int csz = (int)x;
    const int cst = st + (int)off;
    const bool eq = degenerate && gl == 1;
    const bool is_fin = own && !eq && csz >= 2 && csz <= 16;
    const bool is_pend = own && !eq && csz > 16;
    const uint64_t Fm = ballot(is_fin) & gmask;
    const uint64_t Pm = ballot(is_pend) & gmask;
    if (is_fin) {
      const int idx = min(nf + (int)__popcll(Fm & below), GroupLds<K, V, G>::kMaxFin - 1);
      L.fin_st[idx] = (uint16_t)cst;
      L.fin_sz[idx] = (uint16_t)csz;
    }
    if (is_pend) {
      const int idx = min(npn + (int)__popcll(Pm & below), GroupLds<K, V, G>::kMaxPend - 1);
      L.pend_st[cur ^ 1][idx] = (uint16_t)cst;
      L.pend_sz[cur ^ 1][idx] = (uint16_t)csz;
    }
    nf += (int)__popcll(Fm);
    npn += (int)__popcll(Pm);
    // The list sizes are bounded by the array size (disjoint buckets of at
    // least 2, resp. 17, keys); the clamps only keep every loop bounded.
    nf = min(nf, GroupLds<K, V, G>::kMaxFin);
    npn = min(npn, GroupLds<K, V, G>::kMaxPend);
    wave_lds_sync();
  }
}

// Rank-counting sort of the remaining pending buckets (after kLevelCap levels).
template <class K, bool V, int G>
__device__ __forceinline__ void rank_sort_pending(GroupLds<K, V, G>& L, int cur, int np) {
  const int gl = lane_id() % G;
  for (int p = 0; ballot(p < np) != 0ull; ++p) {
    const bool active = p < np;
    const int st = active ? (int)L.pend_st[cur][p] : 0;
    const int sz = active ? (int)L.pend_sz[cur][p] : 0;
    K e[4];
    uint32_t v[4];
    int rank[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      const bool ok = active && i < sz;
      e[s] = ok ? L.key[st + i] : K(0);
      if constexpr (V) v[s] = ok ? L.val[st + i] : 0u;
      rank[s] = 0;
    }
    const int jmax = (int)wave_max((uint32_t)sz);
    for (int j = 0; j < jmax; ++j) {
      const bool in = j < sz;
      const K y = in ? L.key[st + j] : K(0);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int i = gl + G * s;
        rank[s] += (in && (y < e[s] || (y == e[s] && j < i))) ? 1 : 0;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      if (active && i < sz) {
        L.key[st + rank[s]] = e[s];
        if constexpr (V) L.val[st + rank[s]] = v[s];
      }
    }
    wave_lds_sync();
  }
}

// Sorts one array of m keys (0 <= m <= 4G) per G-lane group; every lane of
// the wave must call this (loops are wave-uniform).  gk/gv point at the
// group's array in global memory; keys are XORed with flip on load and store.
template <int F, class K, bool V, int G>
__device__ __forceinline__ void rss_group_sort(GroupLds<K, V, G>& L, K* gk, uint32_t* gv, int m, K flip, int k0) {
  const int lane = lane_id();
  const int gl = lane % G;
  const int gbase = lane - gl;
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);
  (void)gmask;

  // 1. load (coalesced within the group)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    if (i < m) {
      L.key[i] = gk[i] ^ flip;
      if constexpr (V) L.val[i] = gv[i];
    }
  }
  int np = m > 16 ? 1 : 0;
  int nf = (m >= 2 && m <= 16) ? 1 : 0;
  if (gl == 0) {
    if (np) {
      L.pend_st[0][0] = 0;
      L.pend_sz[0][0] = (uint16_t)m;
    }
    if (nf) {
      L.fin_st[0] = 0;
      L.fin_sz[0] = (uint16_t)m;
    }
  }
  wave_lds_sync();

  int cur = 0;
  for (int level = 0; ballot(np > 0) != 0ull; ++level) {
    if (level == kLevelCap) {
      rank_sort_pending(L, cur, np);
      break;
    }
    // sample + network-sorted sample, one lane per pending bucket
    if (gl < np) {
      const int st = L.pend_st[cur][gl];
      const int sz = L.pend_sz[cur][gl];
      K smp[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) smp[t] = L.key[st + ((2 * t + 1) * sz) / 32];
      net_sort<F, 16>(smp);
#pragma unroll
      for (int t = 0; t < 16; ++t) L.sample[gl][t] = smp[t];
    }
    wave_lds_sync();
    const int kk = level == 0 ? k0 : 4;
    int npn = 0;
    if (kk == 16)
      split_level<4>(L, cur, np, nf, npn);
    else if (kk == 8)
      split_level<3>(L, cur, np, nf, npn);
    else
      split_level<2>(L, cur, np, nf, npn);
    np = npn;
    cur ^= 1;
  }

  // finish every bucket of 2..16 keys with a network, one bucket per lane
  for (int base = 0; ballot(base < nf) != 0ull; base += G) {
    const int b = base + gl;
    const bool ok = b < nf;
    const int st = ok ? (int)L.fin_st[b] : 0;
    const int sz = ok ? (int)L.fin_sz[b] : 0;
    const int nmax = (int)wave_max((uint32_t)sz);
    finish_dispatch<F>(L, ok, st, sz, nmax);
  }
  wave_lds_sync();

  // store (coalesced within the group)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    if (i < m) {
      gk[i] = L.key[i] ^ flip;
      if constexpr (V) gv[i] = L.val[i];
    }
  }
  wave_lds_sync();
}

}  // namespace ss
