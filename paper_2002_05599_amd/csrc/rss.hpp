// Register Sample Sort (paper, Section 3) for one array of 17..256 keys,
// executed by a group of G lanes (G = 16, 32 or 64) of a wave.
//
// The array is staged in LDS.  Each level of the recursion handles every
// pending bucket (more than 16 keys) of the array:
//
//   1. sample: a team of lanes per pending bucket picks a*k keys at
//      equidistant positions floor((2t+1)*size/(2ak)), one per lane, and
//      sorts them with a bitonic network laid across the team's lanes (the
//      paper sorts the sample with its base-case sorting network, Section 3;
//      here the network spans lanes instead of one lane's registers).  k
//      buckets with oversampling a = 3 for k = 4 (the paper's "332"), a = 2
//      for k = 8 and a = 1 for k = 16, 32, 64 (the first level may use 32 or
//      64 buckets for arrays of more than 64 or 128 keys; later levels use 4);
//   2. splitters: s_i = S_{a*i} for i = 1..k-1 (Section 3, basic sample
//      sort);
//   3. classify: bucket j = #{splitters < e}, i.e. s_j < e <= s_{j+1}, found
//      by descending the perfect splitter tree without branches: compare with
//      the root, then keep either the left or the right subtree with selects
//      (Section 3 copies one subtree and replaces it by the other only when
//      the comparison says so), and append the comparison bit to the bucket
//      index, j = 2j + [e > root].  The first level holds a narrow
//      tree (at most 32 bytes of splitters) in registers; wider trees and
//      later levels, whose lanes work on different buckets, search the
//      bucket's sorted sample in LDS with the same branch-free steps;
//   4. scatter: a multisplit -- LDS atomic counters give each key its rank
//      within its bucket, per-bucket counts are scanned into offsets -- and
//      the keys are written back in bucket order;
//   5. buckets of 2..16 keys join the finish list, larger ones are pending
//      for the next level (the paper recurses until buckets are at most 16).
//
// Buckets on the finish list are sorted one per lane, by the network of the
// smallest size N covering every bucket of the wave: the lane loads the N keys
// from its bucket's start on.  Buckets lie in key order, so the keys past the
// bucket (later buckets, then the maximum key filling the slack past the
// array) are never smaller than the bucket's own; a compare-exchange between
// a bucket channel and a later channel therefore never swaps (the one-sided
// argument that lets a network of N channels sort fewer keys), channels
// 0..m-1 end sorted, and only they are stored.
//
// Termination with duplicate keys (not covered by the paper): if all k-1
// splitters of a bucket are equal to v, the bucket is split three ways,
// {e < v}, {e == v}, {e > v}; the middle part is already in final order.  Every
// other split sends the smallest splitter's key to bucket 0 and the largest
// splitter's key above it, so every child is strictly smaller than its parent.
// After a cap of levels (kLevelCap, or fewer when tuned down) any remaining
// pending bucket is finished by a rank-counting sort (each key's final
// position is the number of keys that must precede it), which is always
// correct.
#pragma once

#include "common.hpp"

namespace ss {

constexpr int kLevelCap = 8;

// Run-time choices of the recursion: levels before the rank-counting
// fallback (1..kLevelCap), the oversampling factor a of the levels with
// k = 4 buckets (1..4: a sample of 4a keys, splitters at ranks a, 2a, 3a) and
// how buckets are finished (0: networks, 1: rank counting, see
// finish_by_rank).
struct RssCfg {
  int level_cap;
  int a4;
  int finish;
};

template <class K, int V, int G> struct GroupLds {
  static constexpr int kCap = 4 * G;          // keys per array handled by a G-lane group
  static constexpr int kMaxPend = kCap / 17;  // buckets with more than 16 keys
  static constexpr int kMaxFin = kCap / 2;    // buckets with 2..16 keys
  // keys (and values) of the array, plus kPad slack entries holding the
  // maximum key, so that a 16-wide window starting at any bucket of 2 or more
  // keys stays inside the array and reads nothing smaller than the bucket's
  // keys; the last entry, beyond every window, is the sink of the finish
  static constexpr int kPad = 16;
  K key[kCap + kPad];
  Pay<V> val[V ? kCap + kPad : 1];
  // Per pending bucket b, 16 entries from b*16: its sorted sample, the count
  // (then start position) of each child and each child's pending index at the next
  // level (0xFF if none).  The first level has one bucket and may use up to
  // 64 entries (k = 32 or 64 children), which the arrays hold for G >= 32.
  // The rank-counting finish reuses their space for one counter per position.
  union {
    struct {
      K sample[kMaxPend * 16];
      uint32_t cnt[kMaxPend * 16];
    };
    uint32_t tie[kCap];
  };
  uint8_t nextpb[kMaxPend * 16];
  uint8_t deg[kMaxPend];           // all splitters of the bucket equal
  uint8_t pb[kCap];                // pending bucket of each position, or 0xFF
  uint8_t bst[kCap];               // rank-counting finish: start of each position's final bucket
  uint16_t pend_st[2][kMaxPend];
  uint16_t pend_sz[2][kMaxPend];
  uint16_t fin[kMaxFin];            // finish list: start | size << 9 (start < 512, size <= 16)
  static_assert(sizeof(K) * kMaxPend * 16 + 4 * kMaxPend * 16 >= 4 * kCap, "the counters fit the union");
  static_assert(kCap <= 256, "bucket starts are bytes");
};

__device__ __forceinline__ uint16_t fin_pack(int st, int sz) { return (uint16_t)(st | (sz << 9)); }

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

// Finish the buckets of the finish list with networks of N channels: each
// lane reads the N-key window at its bucket's start (the keys past the
// bucket are never smaller, see above) and stores back only the bucket's own
// n channels (the windows reach at most 14 entries past the array; the last
// slack entry is the sink).  Insertion sort, which is not data-oblivious, pads its window
// with the maximum key instead, so that it does no work past the bucket.
template <int F, int N, class K, int V, int G>
__device__ __forceinline__ void finish_buckets(GroupLds<K, V, G>& L, bool ok, int st, int sz) {
  K r[N];
  Pay<V> v[N];
  const int n = ok ? sz : 0;
  K* kp = &L.key[st];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const K x = kp[j];
    r[j] = (F != kFamilyInsertion || j < n) ? x : KeyTraits<K>::kMax;
  }
  Pay<V>* vp = &L.val[V ? st : 0];
  if constexpr (V) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = vp[j];
    net_sort<F, N>(r, v);
  } else {
    net_sort<F, N>(r);
  }
  // channels past the bucket are stored to a sink entry that no window reads
  // (a select of the index keeps the stores unconditional, which the register
  // allocation of the kernels needs)
  constexpr int kSink = GroupLds<K, V, G>::kCap + GroupLds<K, V, G>::kPad - 1;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int dst = j < n ? st + j : kSink;
    L.key[dst] = r[j];
    if constexpr (V) L.val[dst] = v[j];
  }
}

template <int F, class K, int V, int G>
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

// Finish by rank counting (a tuning alternative to the networks): every key
// counts the keys of its final bucket that are smaller than itself, scanning
// N keys from the bucket's start (past the bucket no key is smaller, see
// above), and equal keys take consecutive slots from a counter at their
// common rank.  Each key (and payload) then moves once, where a network
// moves it at every exchange that swaps; for 64-bit keys or payloads, whose
// exchanges take several selects each, that is the cheaper finish.  Keys not
// in a bucket of 2..16 (buckets of one key, runs of equal keys, buckets that
// the fallback sorted) have a bucket start at which they count no smaller
// key, and stay where they are (a run of equal keys permutes within itself).
template <int N, class K, int V, int G>
__device__ __forceinline__ void finish_by_rank(GroupLds<K, V, G>& L, int m) {
  const int gl = lane_id() % G;
#pragma unroll
  for (int s = 0; s < 4; ++s) L.tie[gl + G * s] = 0u;
  wave_lds_sync();
  K e[4];
  Pay<V> v[4];
  int dst[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    dst[s] = -1;
    if (i < m) {
      e[s] = L.key[i];
      if constexpr (V) v[s] = L.val[i];
      const int b = L.bst[i];
      const K* w = &L.key[b];
      int lt = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) lt += (w[j] < e[s]) ? 1 : 0;
      dst[s] = b + lt + (int)atomicAdd(&L.tie[b + lt], 1u);
    }
  }
  wave_lds_sync();  // every key was read before any is written
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (dst[s] >= 0) {
      L.key[dst[s]] = e[s];
      if constexpr (V) L.val[dst[s]] = v[s];
    }
  }
  wave_lds_sync();
}

template <class K, int V, int G>
__device__ __forceinline__ void finish_rank_dispatch(GroupLds<K, V, G>& L, int m, int nmax) {
  switch (nmax) {
    case 2: finish_by_rank<2>(L, m); break;
    case 3: finish_by_rank<3>(L, m); break;
    case 4: finish_by_rank<4>(L, m); break;
    case 5: finish_by_rank<5>(L, m); break;
    case 6: finish_by_rank<6>(L, m); break;
    case 7: finish_by_rank<7>(L, m); break;
    case 8: finish_by_rank<8>(L, m); break;
    case 9: finish_by_rank<9>(L, m); break;
    case 10: finish_by_rank<10>(L, m); break;
    case 11: finish_by_rank<11>(L, m); break;
    case 12: finish_by_rank<12>(L, m); break;
    case 13: finish_by_rank<13>(L, m); break;
    case 14: finish_by_rank<14>(L, m); break;
    case 15: finish_by_rank<15>(L, m); break;
    default: finish_by_rank<16>(L, m); break;
  }
}

// Oversampling factor a for k buckets: the sample of a*k keys must fit one
// network of at most 16 channels.  k = 4 uses a = 3 (12 samples), the
// parameters the paper found best on most machines ("332", Section 4.5).
__host__ __device__ constexpr int oversampling(int k) { return k == 4 ? 3 : (k >= 16 ? 1 : 16 / k); }

// The oversampling a G-lane group uses for k buckets (a4: the tuned factor of
// the 4-bucket levels): an 8-lane group sorts its sample across its 8 lanes,
// so a*k <= 8 there.
__host__ __device__ constexpr int sample_a(int k, int a4, int G) {
  const int a = k == 4 ? a4 : oversampling(k);
  return (G < 16 && a * k > G) ? G / k : a;
}

// Sample team size for k buckets: a power of two holding the a*k samples,
// 16 lanes or the whole group if that is smaller.
__host__ __device__ constexpr int sample_team(int k, int G) {
  return oversampling(k) * k <= 16 ? (G < 16 ? G : 16) : oversampling(k) * k;
}

// Entries per pending bucket in the child counters: one pass of the group's
// lanes scans the children of a bucket.
__host__ __device__ constexpr int child_span(int k, int G) { return G < 16 ? G : (k > 16 ? k : 16); }

// Largest first-level bucket count a G-lane group supports: the first
// level's children are scanned in one pass of the group's lanes, and their
// per-bucket entries must fit the arrays above.
__host__ __device__ constexpr int max_first_k(int G) { return G >= 64 ? 64 : (G >= 32 ? 32 : (G >= 16 ? 16 : 8)); }

// x of lane (lane ^ J), for a compile-time J: DPP for the quad and row
// patterns, a ds_swizzle within 32 lanes otherwise, a lane permute only when
// the partner is in the other half of the wave.  None needs an address
// register.
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x) {
  const int v = (int)x;
  if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);  // quad [1,0,3,2]
  else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
  else if constexpr (J == 3) return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0x1B, 0xF, 0xF, true);  // [3,2,1,0]
  else if constexpr (J == 7) return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // half-row mirror
  else if constexpr (J == 15) return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row mirror
  else if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1F | (J << 10));  // bitmask mode
  else return read_lane(x, lane_id() ^ J);
}

template <int J, class K>
__device__ __forceinline__ K lane_xor_key(K x) {
  if constexpr (sizeof(K) == 8)
    return ((K)lane_xor<J>((uint32_t)(x >> 32)) << 32) | lane_xor<J>((uint32_t)x);
  else
    return lane_xor<J>(x);
}

// Compare-exchange with the lane J apart: the lane whose bit B is clear keeps
// the minimum, the other the maximum.
// (The lower lane takes y if y < x, the upper one if not: with equal keys
// either choice gives the same value, so one compare and one select suffice.)
template <int J, int B, class K>
__device__ __forceinline__ K team_exchange(K x, int t) {
  const K y = lane_xor_key<J>(x);
  const bool upper = (t & B) != 0;
  return ((y < x) != upper) ? y : x;
}

template <int KBLK, int J, class K>
__device__ __forceinline__ K team_half_cleaners(K x, int t) {
  if constexpr (J >= 1) {
    x = team_exchange<J, J>(x, t);
    return team_half_cleaners<KBLK, J / 2>(x, t);
  } else {
    return x;
  }
}

template <int KBLK, int T, class K>
__device__ __forceinline__ K team_merges(K x, int t) {
  if constexpr (KBLK <= T) {
    x = team_exchange<KBLK - 1, KBLK / 2>(x, t);
    x = team_half_cleaners<KBLK, KBLK / 4>(x, t);
    return team_merges<KBLK * 2, T>(x, t);
  } else {
    return x;
  }
}

// Sorts x ascending across each aligned team of T lanes (T a power of two)
// with Batcher's bitonic network in its one-direction form: each merge of
// blocks of size k starts by comparing lane i with its mirror i ^ (k-1) and
// continues with the half-cleaners i ^ j (j = k/4, ..., 1); in every exchange
// the lower lane keeps the minimum.  log T (log T + 1) / 2 exchange stages.
// t = lane index within the team.
template <int T, class K>
__device__ __forceinline__ K team_sort(K x, int t) {
  return team_merges<2, T>(x, t);
}

// Sample of NS = a*k keys (k = KB buckets) at positions
// floor((2t+1)*size/(2*NS)) of each pending bucket (a team of T >= NS lanes
// per bucket, one key per lane, the T - NS spare lanes holding the maximum
// key), sorted across the team; also clears the bucket's child counters and
// records whether all of its k-1 splitters are equal.
template <int KB, int A4, class K, int V, int G>
__device__ __forceinline__ void sample_phase(GroupLds<K, V, G>& L, int cur, int np) {
  // k = 4: the tuned oversampling A4 (a team of 16 lanes holds up to 16 samples)
  constexpr int A = sample_a(KB, A4, G);
  constexpr int NS = A * KB;
  constexpr int T = sample_team(KB, G);  // team size, a power of two
  constexpr int PER = G / T;              // buckets sampled per pass
  constexpr int kSpan = child_span(KB, G);
  static_assert(PER >= 1 && T * PER == G && NS <= T, "team must divide the group and hold the sample");
  const int lane = lane_id();
  const int gl = lane % G;
  const int team = gl / T;
  const int t = gl - team * T;
  for (int b0 = 0; ballot(b0 < np) != 0ull; b0 += PER) {
    const int b = b0 + team;
    const bool own = b < np;
    const int st = own ? (int)L.pend_st[cur][b] : 0;
    const int sz = own ? (int)L.pend_sz[cur][b] : 0;
    K x = KeyTraits<K>::kMax;
    if (own && t < NS) x = L.key[st + ((2 * t + 1) * sz) / (2 * NS)];
    x = team_sort<T>(x, t);
    if (own) {
      if (t < NS) L.sample[b * 16 + t] = x;
      if (t < kSpan) L.cnt[b * kSpan + t] = 0;
    }
    wave_lds_sync();
    // all k-1 splitters equal: the smallest (rank A) equals the largest (rank A*(k-1))
    if (own && t == 0) L.deg[b] = L.sample[b * 16 + A - 1] == L.sample[b * 16 + A * (KB - 1) - 1] ? 1 : 0;
  }
}

// #{i = 1..k-1 : s_i < e} for the splitters s_i = smp[A*i - 1] of a sorted
// sample held in LDS: a branch-free binary search (the in-memory splitter
// tree of super scalar sample sort that the paper's register tree replaces).
template <int LOGK, int A, class K>
__device__ __forceinline__ int lds_bucket(K e, const K* smp) {
  const K* p = smp;  // smp + A*j: each probe is a fixed offset from it
#pragma unroll
  for (int step = (1 << LOGK) / 2; step >= 1; step >>= 1) {
    const K sp = p[A * step - 1];
    p = (sp < e) ? p + A * step : p;
  }
  return (int)(p - smp) / A;
}

// Inclusive sum of x over aligned segments of S lanes (S = 8, 16, 32 or 64):
// Hillis-Steele steps within each row of 16 lanes by row shifts (a lane with
// no source adds 0), then the last lane of a row is broadcast to the next row
// (S >= 32) and lane 31 to the upper half (S = 64), all as DPP operands.
template <int S>
__device__ __forceinline__ uint32_t segment_scan(uint32_t x) {
  static_assert(S == 8 || S == 16 || S == 32 || S == 64, "segments are half rows, rows, row pairs or the wave");
  if constexpr (S == 8) {
    // half rows: the shifts by 1 and 2 would cross from lane 7 of a row to
    // lane 8, so those lanes drop the shifted value; the shift by 4 reaches
    // only the upper four lanes of each half row (banks 1 and 3)
    const int h = lane_id() & 7;
    const uint32_t y1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
    x += h >= 1 ? y1 : 0u;
    const uint32_t y2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
    x += h >= 2 ? y2 : 0u;
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xA, false);  // row_shr:4, banks 1, 3
    return x;
  }
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  if constexpr (S >= 32) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  if constexpr (S >= 64) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// Three-way split of a bucket whose splitters all equal v: {<v}, {==v}, {>v}.
template <class K>
__device__ __forceinline__ int three_way(K e, K v) {
  return e < v ? 0 : (e == v ? 1 : 2);
}

// One level of the recursion for every pending bucket of the group at once
// (k = 2^LOGK children per bucket).  kFirst: the single bucket [0, m) whose
// splitters are held in registers and classified by the register tree; later
// levels take each key's bucket from pb[] and search that bucket's sample in
// LDS.
//
// Multisplit: each key takes its rank among the keys of the same (bucket,
// child) from an LDS atomic counter cnt[b][c] (one ds_add_rtn per key; the
// order of equal-child keys inside a bucket does not matter, because every
// bucket is sorted afterwards).  Per bucket, the counts are scanned into child
// start positions, the children are registered (finish list or next-level
// pending list, in position order) and every key is written to its child's
// start + rank, together with its next-level bucket id when a next level
// follows.
template <int LOGK, bool kFirst, int A4, class K, int V, int G>
__device__ __forceinline__ void split_level(GroupLds<K, V, G>& L, int m, int cur, int np, int& nf, int& npn,
                                            bool track) {
  constexpr int k = 1 << LOGK;
  constexpr int a = sample_a(k, A4, G);
  constexpr int kSpan = child_span(k, G);  // entries per bucket in cnt/nextpb
  static_assert(kFirst || k <= 16, "only the first level has more than 16 children");
  static_assert(kSpan <= G, "the children of a bucket are scanned in one pass");
  const int lane = lane_id();
  const int gl = lane % G;
  const int gbase = lane - gl;
  const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gbase);

  // Level 0 with few, narrow splitters: s_1..s_{k-1} held in registers and
  // searched by the register tree (paper, Section 3).  Wider trees would take
  // more VGPRs than they save and cost occupancy, so they are searched in LDS.
  constexpr bool kRegTree = kFirst && (k - 1) * (int)sizeof(K) <= 32;
  K spl[kRegTree ? k - 1 : 1];
  bool deg0 = false;
  if constexpr (kRegTree) {
#pragma unroll
    for (int i = 0; i < k - 1; ++i) spl[i] = np > 0 ? L.sample[a * (i + 1) - 1] : K(0);
    deg0 = np > 0 && spl[0] == spl[k - 2];
  } else if constexpr (kFirst) {
    deg0 = np > 0 && L.deg[0] != 0;
  }

  // per slot: the key, its payload and where it goes -- the index of its
  // (bucket, child) entry << 16 | its rank among that child's keys, or ~0 if
  // the key is not in a pending bucket.  The slots are handled side by side
  // (loads, then the searches, then the counters), so that the dependent LDS
  // reads of the four searches overlap.
  K e[4];
  Pay<V> v[4];
  uint32_t dst[4];
  int pp[4], cc[4];
  bool dg[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    pp[s] = 0xFF;
    if (i < m) pp[s] = kFirst ? (np > 0 ? 0 : 0xFF) : (int)L.pb[i];
    const bool ok = pp[s] != 0xFF;
    e[s] = ok ? L.key[i] : K(0);
    if constexpr (V) v[s] = ok ? L.val[i] : Pay<V>(0);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if constexpr (kRegTree) {
      cc[s] = classify<LOGK>(e[s], spl);
      dg[s] = deg0;
    } else if constexpr (kFirst) {
      cc[s] = lds_bucket<LOGK, a>(e[s], &L.sample[0]);
      dg[s] = deg0;
    } else {
      const int q = pp[s] != 0xFF ? pp[s] : 0;
      cc[s] = lds_bucket<LOGK, a>(e[s], &L.sample[q * 16]);
      dg[s] = L.deg[q] != 0;
    }
  }
  // buckets whose splitters are all equal split three ways (rare: one
  // wave-uniform test)
  if (ballot(dg[0] || dg[1] || dg[2] || dg[3]) != 0ull) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = pp[s] != 0xFF ? pp[s] : 0;
      const K v0 = kRegTree ? spl[0] : L.sample[q * 16 + a - 1];
      if (dg[s]) cc[s] = three_way(e[s], v0);
    }
  }
  // rank among the keys of the same (bucket, child): an LDS atomic counter
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int ci = pp[s] * kSpan + cc[s];
    dst[s] = ~0u;
    if (pp[s] != 0xFF) dst[s] = ((uint32_t)ci << 16) | atomicAdd(&L.cnt[ci], 1u);
  }
  wave_lds_sync();

  // scan each bucket's child counts into offsets; register the children
  for (int r0 = 0; ballot(r0 < np * kSpan) != 0ull; r0 += G) {
    const int q = r0 + gl;
    const int pq = q / kSpan;
    const int cq = q % kSpan;
    const bool okq = pq < np;
    const bool dg = okq && L.deg[pq] != 0;
    const int nchq = okq ? (dg ? 3 : k) : 0;
    const bool own = cq < nchq;
    const uint32_t x = own ? L.cnt[q] : 0u;
    const uint32_t off = segment_scan<kSpan>(x) - x;
    const int cst = okq ? (int)L.pend_st[cur][pq] + (int)off : 0;
    const int csz = (int)x;
    const bool eq = dg && cq == 1;
    const bool is_fin = own && !eq && csz >= 2 && csz <= 16;
    const bool is_pend = own && !eq && csz > 16;
    const uint64_t Fm = ballot(is_fin) & gmask;
    const uint64_t Pm = ballot(is_pend) & gmask;
    if (own) L.cnt[q] = (uint32_t)cst;
    if (is_fin) {
      const int idx = min(nf + (int)mbcnt(Fm), GroupLds<K, V, G>::kMaxFin - 1);
      L.fin[idx] = fin_pack(cst, csz);
    }
    int pidx = 0xFF;
    if (is_pend) {
      pidx = min(npn + (int)mbcnt(Pm), GroupLds<K, V, G>::kMaxPend - 1);
      L.pend_st[cur ^ 1][pidx] = (uint16_t)cst;
      L.pend_sz[cur ^ 1][pidx] = (uint16_t)csz;
    }
    if (own) L.nextpb[q] = (uint8_t)pidx;
    // The list sizes are bounded by the array size (disjoint buckets of at
    // least 2, resp. 17, keys); the clamps only keep every loop bounded.
    nf = min(nf + (int)__popcll(Fm), GroupLds<K, V, G>::kMaxFin);
    npn = min(npn + (int)__popcll(Pm), GroupLds<K, V, G>::kMaxPend);
  }
  wave_lds_sync();

  // scatter in place (every key of the slots was read above); the next-level
  // bucket ids are needed only if some group of the wave has a next level
  const bool more = ballot(npn > 0) != 0ull;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (dst[s] != ~0u) {
      const int pc = (int)(dst[s] >> 16);
      const int cst = (int)L.cnt[pc];
      const int pos = cst + (int)(dst[s] & 0xFFFFu);
      L.key[pos] = e[s];
      if constexpr (V) L.val[pos] = v[s];
      if (more) L.pb[pos] = L.nextpb[pc];
      if (track) L.bst[pos] = (uint8_t)cst;
    }
  }
  wave_lds_sync();
}

// One level with k = 4 buckets and the tuned oversampling a4 (each a
// compile-time variant: a run-time factor costs registers in every level).
template <int A4, bool kFirst, class K, int V, int G>
__device__ __forceinline__ void level_k4_a(GroupLds<K, V, G>& L, int m, int cur, int np, int& nf, int& npn,
                                           bool track) {
  sample_phase<4, A4>(L, cur, np);
  wave_lds_sync();
  split_level<2, kFirst, A4>(L, m, cur, np, nf, npn, track);
}
template <bool kFirst, class K, int V, int G>
__device__ __forceinline__ void level_k4(GroupLds<K, V, G>& L, int m, int cur, int np, int& nf, int& npn, int a4,
                                         bool track) {
  switch (a4) {
    case 1: level_k4_a<1, kFirst>(L, m, cur, np, nf, npn, track); break;
    case 2: level_k4_a<2, kFirst>(L, m, cur, np, nf, npn, track); break;
    case 4: level_k4_a<4, kFirst>(L, m, cur, np, nf, npn, track); break;
    default: level_k4_a<3, kFirst>(L, m, cur, np, nf, npn, track); break;
  }
}

// Rank-counting sort of the remaining pending buckets (after kLevelCap levels).
template <class K, int V, int G>
__device__ __forceinline__ void rank_sort_pending(GroupLds<K, V, G>& L, int cur, int np, bool track) {
  const int gl = lane_id() % G;
  for (int p = 0; ballot(p < np) != 0ull; ++p) {
    const bool active = p < np;
    const int st = active ? (int)L.pend_st[cur][p] : 0;
    const int sz = active ? (int)L.pend_sz[cur][p] : 0;
    K e[4];
    Pay<V> v[4];
    int rank[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = gl + G * s;
      const bool ok = active && i < sz;
      e[s] = ok ? L.key[st + i] : K(0);
      if constexpr (V) v[s] = ok ? L.val[st + i] : Pay<V>(0);
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
        if (track) L.bst[st + rank[s]] = (uint8_t)(st + rank[s]);  // in final place: a bucket of its own
      }
    }
    wave_lds_sync();
  }
}

// Sorts the array of m keys (0 <= m <= 4G) that the group holds in L.key (and
// L.val), in place in LDS.  Every lane of the wave must call this (loops are
// wave-uniform).  k0: first-level bucket count; level_cap (1..kLevelCap):
// levels of sample sort before the rank-counting fallback.
template <int F, class K, int V, int G>
__device__ __forceinline__ void rss_group_sort_lds(GroupLds<K, V, G>& L, int m, int k0, RssCfg cfg) {
  const int gl = lane_id() % G;
  const bool track = cfg.finish != 0;  // record each position's final bucket (rank-counting finish)
  int np = m > 16 ? 1 : 0;
  int nf = (m >= 2 && m <= 16) ? 1 : 0;
  // the slack past the array holds the maximum key; an array of at most 16
  // keys is one bucket (its final-bucket starts are 0)
#pragma unroll
  for (int t = 0; t < GroupLds<K, V, G>::kPad; t += G)
    if (t + gl < GroupLds<K, V, G>::kPad) L.key[m + t + gl] = KeyTraits<K>::kMax;
  if (track) {
#pragma unroll
    for (int t = 0; t < 16; t += G)
      if (t + gl < 16) L.bst[t + gl] = 0;
  }
  if (gl == 0) {
    if (np) {
      L.pend_st[0][0] = 0;
      L.pend_sz[0][0] = (uint16_t)m;
    }
    if (nf) L.fin[0] = fin_pack(0, m);
  }
  wave_lds_sync();

  int cur = 0;
  for (int level = 0; ballot(np > 0) != 0ull; ++level) {
    if (level == cfg.level_cap) {
      rank_sort_pending(L, cur, np, track);
      break;
    }
    const int kk = level == 0 ? min(k0, max_first_k(G)) : 4;
    int npn = 0;
    if (kk == 64) {
      if constexpr (max_first_k(G) >= 64) {
        sample_phase<64, 3>(L, cur, np);
        wave_lds_sync();
        split_level<6, true, 3>(L, m, cur, np, nf, npn, track);
      }
    } else if (kk == 32) {
      if constexpr (max_first_k(G) >= 32) {
        sample_phase<32, 3>(L, cur, np);
        wave_lds_sync();
        split_level<5, true, 3>(L, m, cur, np, nf, npn, track);
      }
    } else if (kk == 16) {
      if constexpr (max_first_k(G) >= 16) {
        sample_phase<16, 3>(L, cur, np);
        wave_lds_sync();
        split_level<4, true, 3>(L, m, cur, np, nf, npn, track);
      }
    } else if (kk == 8) {
      sample_phase<8, 3>(L, cur, np);
      wave_lds_sync();
      split_level<3, true, 3>(L, m, cur, np, nf, npn, track);
    } else if (level == 0) {
      level_k4<true>(L, m, cur, np, nf, npn, cfg.a4, track);
    } else {
      level_k4<false>(L, m, cur, np, nf, npn, cfg.a4, track);
    }
    np = npn;
    cur ^= 1;
  }

  if (track) {
    // the largest bucket of the wave's finish lists bounds every window
    int nmax = 0;
    for (int b = gl; b < nf; b += G) nmax = max(nmax, (int)(L.fin[b] >> 9));
    nmax = (int)wave_max((uint32_t)nmax);
    if (nmax >= 2) finish_rank_dispatch(L, m, nmax);
    return;
  }
  // finish every bucket of 2..16 keys with a network, one bucket per lane
  for (int base = 0; ballot(base < nf) != 0ull; base += G) {
    const int b = base + gl;
    const bool ok = b < nf;
    const int fe = ok ? (int)L.fin[b] : 0;
    const int st = fe & 511;
    const int sz = fe >> 9;
    const int nmax = (int)wave_max((uint32_t)sz);
    finish_dispatch<F>(L, ok, st, sz, nmax);
  }
  wave_lds_sync();
}

// Global -> LDS (keys XORed with flip), coalesced within the group.
template <class K, int V, int G>
__device__ __forceinline__ void rss_group_load(GroupLds<K, V, G>& L, const K* gk, const Pay<V>* gv, int m, KeyMap<K> flip) {
  const int gl = lane_id() % G;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    if (i < m) {
      L.key[i] = flip.enc(gk[i]);
      if constexpr (V) L.val[i] = gv[i];
    }
  }
}

// LDS -> global (keys XORed with flip), coalesced within the group.
template <class K, int V, int G>
__device__ __forceinline__ void rss_group_store(GroupLds<K, V, G>& L, K* gk, Pay<V>* gv, int m, KeyMap<K> flip) {
  const int gl = lane_id() % G;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int i = gl + G * s;
    if (i < m) {
      gk[i] = flip.dec(L.key[i]);
      if constexpr (V) gv[i] = L.val[i];
    }
  }
}

// Loads, sorts and stores one array of m keys per G-lane group; gk/gv point at
// the group's array in global memory; keys are XORed with flip on load and
// store.
template <int F, class K, int V, int G>
__device__ __forceinline__ void rss_group_sort(GroupLds<K, V, G>& L, K* gk, Pay<V>* gv, int m, KeyMap<K> flip, int k0,
                                               RssCfg cfg) {
  rss_group_load(L, gk, gv, m, flip);
  wave_lds_sync();
  rss_group_sort_lds<F>(L, m, k0, cfg);
  rss_group_store(L, gk, gv, m, flip);
  wave_lds_sync();
}

}  // namespace ss
