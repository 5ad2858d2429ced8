// Sorting one large array on the device with the small sorters as its base
// case (the paper's Section 4.4 and 4.6 integrations into Quicksort and
// IPS4o, and Section 5's proposal to sort the base cases in batches grouped
// by size).
//
// One level is a sample sort partition of the whole array:
//   sample    16k keys at hashed positions, sorted by this same sort (or by
//             the small sorters when the sample has at most 4096 keys);
//   splitters every 16th sample key: k - 1 splitters s_0 <= ... <= s_{k-2};
//   classify  a key e goes to bucket 2j, j = #{splitters < e}, or to the
//             equality bucket 2j + 1 when e == s_j (IPS4o's equality
//             buckets: a value that fills several splitters lands in one
//             bucket that needs no sorting); branch-free binary searches,
//             first over every 256th splitter held in LDS, then inside
//             the block of 256 splitters it selects;
//   count     one atomic counter per bucket; an exclusive scan gives the
//             bucket offsets;
//   scatter   every key (and payload) to its bucket in the temporary buffer.
// A level of more than kDsTwoPassBlocks blocks of splitters (about two million
// keys and up) moves the keys in two passes instead, without one global
// atomic per key: the first search step alone (the block h of 256 splitters
// a key falls in, an LDS search) orders the keys by block -- per work-group
// histograms in LDS, one atomic per block and work-group to reserve its
// ranges, the keys scattered to the temporary buffer -- and then one
// work-group per block stages the block's splitters in LDS, counts and
// scatters its keys to their buckets in the caller's buffer and writes the
// block's bucket offsets.
// The buckets are then the segments of one segmented sort (networks, Register
// Sample Sort, the work-group sort up to 4096 keys), k is chosen so that a
// bucket holds about 1536 keys of 4 bytes or 1024 of 8 (ds_per_bucket).  A range bucket that still holds more than
// 4096 keys is sorted by the same algorithm, recursively, with the other
// buffer as its temporary; equality buckets are left as they are.  Finally
// the buckets are copied back where the single-pass partition left them in
// the temporary buffer.
//
// The host reads two numbers per level (the count of oversized buckets and
// their bounds), so the call synchronises its stream; it allocates nothing
// (all working memory is carved from the caller's workspace).
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace ss {

constexpr int kDsThreads = 256;
constexpr int64_t kDsBaseN = 4096;   // largest bucket the segmented sort takes
// target mean bucket size: 1536 keys of 4 bytes, 1024 of 8 (on 2^28 uint32
// keys 1536 measured 10% faster than 1024, on 2^26 uint64 keys 9% slower;
// 2048 sends too many buckets above 4096 keys to another level)
__host__ __device__ constexpr int64_t ds_per_bucket(size_t key_bytes) { return key_bytes == 4 ? 1536 : 1024; }
constexpr int kDsOversample = 16;
constexpr int kDsMaxSplitters = (1 << 20) - 1;

__device__ __forceinline__ uint64_t ds_mix(uint64_t z) {  // SplitMix64 output function
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// sample[t] = keys[hash(t) mod n]
template <class K>
__global__ void __launch_bounds__(kDsThreads)
ds_sample_kernel(const K* __restrict__ keys, int64_t n, K* __restrict__ sample, int64_t s, uint64_t seed) {
  for (int64_t t = (int64_t)blockIdx.x * kDsThreads + threadIdx.x; t < s; t += (int64_t)gridDim.x * kDsThreads)
    sample[t] = keys[ds_mix(seed + (uint64_t)t * 0x9E3779B97F4A7C15ull) % (uint64_t)n];
}

// splitter i = sorted sample word [16 i + 8], i < nspl
template <class K>
__global__ void __launch_bounds__(kDsThreads)
ds_splitter_kernel(const K* __restrict__ sorted_sample, K* __restrict__ spl, int nspl, KeyMap<K> map) {
  for (int i = blockIdx.x * kDsThreads + threadIdx.x; i < nspl; i += gridDim.x * kDsThreads)
    spl[i] = map.enc(sorted_sample[(int64_t)i * kDsOversample + kDsOversample / 2]);
}

// The splitter search in two steps: the last splitter of every block of
// kDsBlock splitters is held in LDS (at most kDsTop of them), a binary search
// there gives the block, a second one inside the block (a few cache lines of
// global memory) gives j.
constexpr int kDsBlock = 256;
constexpr int kDsTop = (kDsMaxSplitters + kDsBlock) / kDsBlock;  // 4096

template <class K>
__device__ __forceinline__ int ds_load_top(K* top, const K* __restrict__ spl, int nspl) {
  const int nt = (nspl + kDsBlock - 1) / kDsBlock;
  for (int t = threadIdx.x; t < nt; t += kDsThreads) top[t] = spl[min((t + 1) * kDsBlock, nspl) - 1];
  __syncthreads();
  return nt;
}

// largest power of two <= x (x >= 1)
__device__ __forceinline__ int ds_pow2_floor(int x) { return 1 << (31 - __builtin_clz((unsigned)x)); }

// blocks whose last splitter is below word e (all their splitters are): 0..nt
template <class K>
__device__ __forceinline__ int ds_top(K e, const K* top, int nt) {
  int tb = 0;
  for (int step = ds_pow2_floor(nt); step >= 1; step >>= 1)
    if (tb + step <= nt && top[tb + step - 1] < e) tb += step;
  return tb;
}

// bucket of word e: 2j or 2j + 1 with j = #{splitters < e} (see above)
template <class K>
__device__ __forceinline__ int ds_bucket(K e, const K* top, int nt, const K* __restrict__ spl, int nspl) {
  const int tb = ds_top(e, top, nt);
  int j = min(tb * kDsBlock, nspl);  // every splitter is below e when tb == nt
  if (tb < nt) {
    const int len = min(kDsBlock, nspl - j);
    int r = 0;
    for (int step = kDsBlock / 2; step >= 1; step >>= 1)
      if (r + step <= len && spl[j + r + step - 1] < e) r += step;
    j += r;
  }
  return 2 * j + ((j < nspl && spl[j] == e) ? 1 : 0);
}

template <class K>
__global__ void __launch_bounds__(kDsThreads)
ds_count_kernel(const K* __restrict__ keys, int64_t n, const K* __restrict__ spl, int nspl,
                uint32_t* __restrict__ counts, KeyMap<K> map) {
  __shared__ K top[kDsTop];
  const int nt = ds_load_top(top, spl, nspl);
  for (int64_t i = (int64_t)blockIdx.x * kDsThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDsThreads)
    atomicAdd(&counts[ds_bucket(map.enc(keys[i]), top, nt, spl, nspl)], 1u);
}

// One work-group: exclusive scan of the bucket counts into offsets[0..nb]
// (int32, the segmented sort's CSR), cursors = offsets; lists the range
// buckets of more than kDsBaseN keys (their index) after counting them.
__global__ void __launch_bounds__(1024)
ds_scan_kernel(const uint32_t* __restrict__ counts, int nb, int32_t* __restrict__ offsets,
               uint32_t* __restrict__ cursors, uint32_t* __restrict__ big, uint32_t* __restrict__ nbig) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = t * per, b1 = min(nb, b0 + per);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += counts[b];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the partial sums
    const uint32_t y = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (int b = b0; b < b1; ++b) {
    offsets[b] = (int32_t)run;
    cursors[b] = run;
    const uint32_t c = counts[b];
    if ((b & 1) == 0 && c > (uint32_t)kDsBaseN) big[atomicAdd(nbig, 1u)] = (uint32_t)b;
    run += c;
  }
  if (t == 1023) offsets[nb] = (int32_t)part[1023];
}

template <class K, int V>
__global__ void __launch_bounds__(kDsThreads)
ds_scatter_kernel(const K* __restrict__ keys, const Pay<V>* __restrict__ vals, int64_t n,
                  const K* __restrict__ spl, int nspl, uint32_t* __restrict__ cursors,
                  K* __restrict__ out_keys, Pay<V>* __restrict__ out_vals, KeyMap<K> map) {
  __shared__ K top[kDsTop];
  const int nt = ds_load_top(top, spl, nspl);
  for (int64_t i = (int64_t)blockIdx.x * kDsThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDsThreads) {
    const K x = keys[i];
    const uint32_t pos = atomicAdd(&cursors[ds_bucket(map.enc(x), top, nt, spl, nspl)], 1u);
    out_keys[pos] = x;
    if constexpr (V) out_vals[pos] = vals[i];
  }
}

// --- the two-pass partition ---------------------------------------------------
//
// Keys are first ordered by their splitter block h = ds_top (0..nt; h = nt
// holds the keys above every splitter), then within each block by bucket.
// Block h < nt covers buckets 2 h 256 .. 2 (h 256 + len) - 1 (len = its
// splitters); block nt covers the last range bucket 2 nspl alone.  A key of
// block h < nt is not above the block's last splitter, so its search inside
// the block ends on a splitter of the block.
constexpr int kDsTwoPassBlocks = 8;

// Keys per work-group of the first pass (a contiguous chunk each).
__device__ __forceinline__ void ds_chunk(int64_t n, int64_t& i0, int64_t& i1) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  i0 = (int64_t)blockIdx.x * chunk;
  i1 = min(n, i0 + chunk);
}

// Calls f(i, key, block) for the keys i0 <= i < i1, kDsUnroll per thread at
// a time: their searches are independent chains of LDS reads that overlap.
constexpr int kDsUnroll = 16;  // (4: 4% slower, 8: 3% slower on 2^28 uint32 keys)
template <class K, class F>
__device__ __forceinline__ void ds_for_blocks(const K* __restrict__ keys, int64_t i0, int64_t i1, const K* top,
                                              int nt, KeyMap<K> map, F f) {
  for (int64_t base = i0 + threadIdx.x; base < i1; base += (int64_t)kDsUnroll * kDsThreads) {
    K x[kDsUnroll];
    int h[kDsUnroll];
#pragma unroll
    for (int u = 0; u < kDsUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kDsThreads;
      x[u] = i < i1 ? keys[i] : K(0);
    }
    // the searches step by step side by side (ds_top for each key)
    K e[kDsUnroll];
#pragma unroll
    for (int u = 0; u < kDsUnroll; ++u) {
      e[u] = map.enc(x[u]);
      h[u] = 0;
    }
    for (int step = ds_pow2_floor(nt); step >= 1; step >>= 1) {
#pragma unroll
      for (int u = 0; u < kDsUnroll; ++u)
        if (h[u] + step <= nt && top[h[u] + step - 1] < e[u]) h[u] += step;
    }
#pragma unroll
    for (int u = 0; u < kDsUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kDsThreads;
      if (i < i1) f(i, x[u], h[u]);
    }
  }
}

// hist[h] = keys of this work-group's chunk in block h (nt + 1 entries)
template <class K>
__device__ __forceinline__ void ds_block_hist(const K* __restrict__ keys, int64_t i0, int64_t i1, const K* top,
                                              int nt, uint32_t* hist, KeyMap<K> map) {
  for (int h = threadIdx.x; h <= nt; h += kDsThreads) hist[h] = 0;
  __syncthreads();
  ds_for_blocks(keys, i0, i1, top, nt, map, [&](int64_t, K, int h) { atomicAdd(&hist[h], 1u); });
  __syncthreads();
}

template <class K>
__global__ void __launch_bounds__(kDsThreads)
ds_block_count_kernel(const K* __restrict__ keys, int64_t n, const K* __restrict__ spl, int nspl,
                      uint32_t* __restrict__ block_count, KeyMap<K> map) {
  __shared__ K top[kDsTop];
  __shared__ uint32_t hist[kDsTop + 1];
  const int nt = ds_load_top(top, spl, nspl);
  int64_t i0, i1;
  ds_chunk(n, i0, i1);
  ds_block_hist(keys, i0, i1, top, nt, hist, map);
  for (int h = threadIdx.x; h <= nt; h += kDsThreads)
    if (hist[h]) atomicAdd(&block_count[h], hist[h]);
}

// One work-group: block_off[0..nb] = exclusive scan of block_count[0..nb),
// block_cursor = block_off (nb <= kDsTop + 1).
__global__ void __launch_bounds__(1024)
ds_block_scan_kernel(const uint32_t* __restrict__ block_count, int nb, uint32_t* __restrict__ block_off,
                     uint32_t* __restrict__ block_cursor) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += block_count[b];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint32_t y = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (int b = b0; b < b1; ++b) {
    block_off[b] = run;
    block_cursor[b] = run;
    run += block_count[b];
  }
  if (t == 1023) block_off[nb] = part[1023];
}

// Keys (and payloads) of each chunk to their blocks' ranges in the temporary
// buffer: the work-group reserves one range per block with one atomic, then
// each key takes the next slot of its block's range (an LDS atomic).
template <class K, int V>
__global__ void __launch_bounds__(kDsThreads)
ds_block_scatter_kernel(const K* __restrict__ keys, const Pay<V>* __restrict__ vals, int64_t n,
                        const K* __restrict__ spl, int nspl, uint32_t* __restrict__ block_cursor,
                        K* __restrict__ out_keys, Pay<V>* __restrict__ out_vals, KeyMap<K> map) {
  __shared__ K top[kDsTop];
  __shared__ uint32_t hist[kDsTop + 1];
  const int nt = ds_load_top(top, spl, nspl);
  int64_t i0, i1;
  ds_chunk(n, i0, i1);
  ds_block_hist(keys, i0, i1, top, nt, hist, map);
  for (int h = threadIdx.x; h <= nt; h += kDsThreads)
    if (hist[h]) hist[h] = atomicAdd(&block_cursor[h], hist[h]);
  __syncthreads();
  ds_for_blocks(keys, i0, i1, top, nt, map, [&](int64_t i, K x, int h) {
    const uint32_t pos = atomicAdd(&hist[h], 1u);
    out_keys[pos] = x;
    if constexpr (V) out_vals[pos] = vals[i];
  });
}

// Work-group h: the keys of block h (block_off[h] .. block_off[h + 1] of the
// temporary buffer) to their buckets in keys/vals; writes offsets[b] for the
// block's buckets (and offsets[nb] = n) and lists its range buckets above
// kDsBaseN keys.
template <class K, int V>
__global__ void __launch_bounds__(kDsThreads)
ds_block_bucket_kernel(const K* __restrict__ tk, const Pay<V>* __restrict__ tv, const K* __restrict__ spl, int nspl,
                       const uint32_t* __restrict__ block_off, K* __restrict__ keys, Pay<V>* __restrict__ vals,
                       int32_t* __restrict__ offsets, int nb, uint32_t* __restrict__ big,
                       uint32_t* __restrict__ nbig, KeyMap<K> map) {
  __shared__ K bs[kDsBlock];
  __shared__ uint32_t cnt[2 * kDsBlock];
  __shared__ uint32_t part[kDsThreads];
  const int nt = (nspl + kDsBlock - 1) / kDsBlock;
  const int h = blockIdx.x;
  const int j0 = h * kDsBlock;
  const int len = h < nt ? min(kDsBlock, nspl - j0) : 0;
  const int nloc = h < nt ? 2 * len : 1;  // buckets of this block
  const int b0 = h < nt ? 2 * j0 : nb - 1;
  const uint32_t lo = block_off[h], hi = block_off[h + 1];
  for (int t = threadIdx.x; t < len; t += kDsThreads) bs[t] = spl[j0 + t];  // splitters are stored as words
  for (int t = threadIdx.x; t < 2 * kDsBlock; t += kDsThreads) cnt[t] = 0;
  __syncthreads();
  // f(i, key, local bucket) for the block's keys: local bucket 2r or 2r + 1,
  // r = #{block splitters < e} (< len, see above); kDsUnroll keys per thread
  // at a time, so that their searches overlap
  auto for_local = [&](auto f) __attribute__((always_inline)) {
    for (uint32_t base = lo + threadIdx.x; base < hi; base += kDsUnroll * kDsThreads) {
      K x[kDsUnroll];
      int lb[kDsUnroll];
#pragma unroll
      for (int u = 0; u < kDsUnroll; ++u) {
        const uint32_t i = base + u * kDsThreads;
        x[u] = i < hi ? tk[i] : K(0);
      }
      // the searches step by step side by side (local for each key)
      K e[kDsUnroll];
      int r[kDsUnroll];
#pragma unroll
      for (int u = 0; u < kDsUnroll; ++u) {
        e[u] = map.enc(x[u]);
        r[u] = 0;
      }
#pragma unroll
      for (int step = kDsBlock / 2; step >= 1; step >>= 1) {
#pragma unroll
        for (int u = 0; u < kDsUnroll; ++u)
          if (r[u] + step <= len && bs[r[u] + step - 1] < e[u]) r[u] += step;
      }
#pragma unroll
      for (int u = 0; u < kDsUnroll; ++u) {
        const int q = max(0, min(r[u], len - 1));  // (r < len already for every key of the block)
        lb[u] = len == 0 ? 0 : 2 * q + (bs[q] == e[u] ? 1 : 0);
      }
#pragma unroll
      for (int u = 0; u < kDsUnroll; ++u) {
        const uint32_t i = base + u * kDsThreads;
        if (i < hi) f(i, x[u], lb[u]);
      }
    }
  };
  for_local([&](uint32_t, K, int b) { atomicAdd(&cnt[b], 1u); });
  __syncthreads();
  // exclusive scan of cnt[0 .. 2 kDsBlock): two entries per thread
  const int t = threadIdx.x;
  const uint32_t c0 = cnt[2 * t], c1 = cnt[2 * t + 1];
  part[t] = c0 + c1;
  __syncthreads();
  for (int d = 1; d < kDsThreads; d <<= 1) {
    const uint32_t y = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  const uint32_t e0 = part[t] - c0 - c1;
  __syncthreads();  // every count is read before the cursors overwrite them
  const uint32_t starts[2] = {e0, e0 + c0}, counts[2] = {c0, c1};
  for (int q = 0; q < 2; ++q) {
    const int lb = 2 * t + q;
    if (lb < nloc) {
      const int b = b0 + lb;
      offsets[b] = (int32_t)(lo + starts[q]);
      if ((b & 1) == 0 && counts[q] > (uint32_t)kDsBaseN) big[atomicAdd(nbig, 1u)] = (uint32_t)b;
    }
    cnt[lb] = starts[q];
  }
  if (h == nt && t == 0) offsets[nb] = (int32_t)hi;
  __syncthreads();
  for_local([&](uint32_t i, K x, int b) {
    const uint32_t pos = lo + atomicAdd(&cnt[b], 1u);
    keys[pos] = x;
    if constexpr (V) vals[pos] = tv[i];
  });
}

template <class K, int V>
__global__ void __launch_bounds__(kDsThreads)
ds_copy_kernel(K* __restrict__ dk, Pay<V>* __restrict__ dv, const K* __restrict__ sk, const Pay<V>* __restrict__ sv,
               int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kDsThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDsThreads) {
    dk[i] = sk[i];
    if constexpr (V) dv[i] = sv[i];
  }
}

// --- workspace ---------------------------------------------------------------

static size_t ds_align(size_t x) { return (x + 255) & ~(size_t)255; }

struct DsPlan {
  int64_t n;
  int nspl;      // k - 1 splitters
  int nb;        // 2k - 1 buckets
  int64_t s;     // sample keys
};

static DsPlan ds_plan(int64_t n, size_t key_bytes) {
  DsPlan p;
  p.n = n;
  const int64_t per = ds_per_bucket(key_bytes);
  int64_t k = (n + per - 1) / per;
  if (k < 2) k = 2;
  if (k - 1 > kDsMaxSplitters) k = kDsMaxSplitters + 1;
  p.nspl = (int)(k - 1);
  p.nb = (int)(2 * k - 1);
  p.s = k * kDsOversample;
  return p;
}

// Working memory of one level for n keys of ksz bytes (besides the n-item
// temporary buffer), including what sorting its sample needs.  The range
// buckets above 4096 keys are sorted afterwards in the same memory: their
// levels are smaller, since the plan grows with n.
static size_t ds_level_bytes(int64_t n, size_t ksz) {
  if (n <= kDsBaseN) return 16384 + kSegHistBytes;  // one segment through the segmented path
  const DsPlan p = ds_plan(n, ksz);
  size_t b = ds_align((size_t)p.s * ksz);                                    // sample
  b += ds_align((size_t)p.nspl * ksz);                                       // splitters
  b += 3 * ds_align((size_t)(p.nb + 1) * 4);                                 // counts, offsets, cursors
  b += ds_align((size_t)(p.nb + 1) * 4) + 256;                               // big-bucket list + count
  b += 3 * ds_align((size_t)(kDsTop + 2) * 4);                               // block counts, offsets, cursors
  b += ds_align((size_t)p.nb * 4) + ds_align(kSegCtrlBytes) + ds_align(kSegHistBytes);  // segmented-sort buffers
  b += ds_align((size_t)p.s * ksz) + ds_level_bytes(p.s, ksz);              // sorting the sample
  return b;
}

struct DsCarve {
  unsigned char* p;
  unsigned char* end;
  void* take(size_t bytes) {
    void* r = p;
    p += ds_align(bytes);
    return p <= end ? r : nullptr;
  }
};

// The small sorters on one array of n <= kDsBaseN keys (count = 1).
template <class K>
static hipError_t ds_small(K* keys, int64_t n, KeyMap<K> map, DeviceCtx* c, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  if constexpr (sizeof(K) == 4) {
    if (n <= 16) return launch_fixed_u32(keys, (int)n, 1, n, map, s);
    if (n <= 256) return launch_rss_fixed_u32(keys, (int)n, 1, n, map, c->status, s);
    return launch_large_fixed_u32(keys, (int)n, 1, n, map, s);
  } else {
    if (n <= 16) return launch_fixed_u64(keys, (int)n, 1, n, map, s);
    if (n <= 256) return launch_rss_fixed_u64(keys, (int)n, 1, n, map, c->status, s);
    return launch_large_fixed_u64(keys, (int)n, 1, n, map, s);
  }
}

template <class K>
static int ds_segmented(DeviceCtx* c, const SegBuffers& b, K* keys, void* vals, int vb, const int32_t* off,
                        int32_t nseg, KeyMap<K> map, hipStream_t s) {
  if constexpr (sizeof(K) == 4)
    return segmented_direct_u32(c, b, keys, vals, vb, off, nseg, map, s);
  else
    return segmented_direct_u64(c, b, keys, vals, vb, off, nseg, map, s);
}

static unsigned ds_grid(DeviceCtx* c, int64_t n) {
  const int64_t want = (n + kDsThreads - 1) / kDsThreads;
  const int64_t cap = (int64_t)c->num_cus * 16;
  return (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
}

// Sorts keys[0, n) (and vals) using tmp_keys/tmp_vals (n items) and the
// workspace [ws, ws_end); the result ends in keys.  depth bounds the recursion.
template <class K, int V>
static hipError_t ds_sort(DeviceCtx* c, K* keys, Pay<V>* vals, int64_t n, K* tmp_keys, Pay<V>* tmp_vals,
                          unsigned char* ws, unsigned char* ws_end, KeyMap<K> map, hipStream_t s, int depth) {
  if (n <= kDsBaseN) {
    if constexpr (V == 0) {
      return ds_small<K>(keys, n, map, c, s);
    } else {
      // one segment [0, n) through the segmented path (it carries payloads)
      if (n <= 1) return hipSuccess;
      DsCarve cv{ws, ws_end};
      auto* off = static_cast<int32_t*>(cv.take(8));
      SegBuffers b;
      b.ids = static_cast<int32_t*>(cv.take(256));
      b.ctrl = static_cast<uint32_t*>(cv.take(kSegCtrlBytes));
      b.blockhist = static_cast<uint32_t*>(cv.take(kSegHistBytes));
      if (!b.blockhist) return hipErrorInvalidValue;
      const int32_t host_off[2] = {0, (int32_t)n};
      hipError_t e = hipMemcpyAsync(off, host_off, sizeof host_off, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(s);  // host_off lives on this stack frame
      if (e != hipSuccess) return e;
      return ds_segmented<K>(c, b, keys, vals, V, off, 1, map, s) == 0 ? hipSuccess : hipErrorUnknown;
    }
  }
  if (depth > 32) return hipErrorUnknown;  // each level splits off at least the equality of a splitter
  const DsPlan p = ds_plan(n, sizeof(K));
  DsCarve cv{ws, ws_end};
  auto* sample = static_cast<K*>(cv.take((size_t)p.s * sizeof(K)));
  auto* spl = static_cast<K*>(cv.take((size_t)p.nspl * sizeof(K)));
  auto* counts = static_cast<uint32_t*>(cv.take((size_t)(p.nb + 1) * 4));
  auto* offsets = static_cast<int32_t*>(cv.take((size_t)(p.nb + 1) * 4));
  auto* cursors = static_cast<uint32_t*>(cv.take((size_t)(p.nb + 1) * 4));
  auto* big = static_cast<uint32_t*>(cv.take((size_t)(p.nb + 1) * 4));
  auto* nbig = static_cast<uint32_t*>(cv.take(256));
  auto* block_count = static_cast<uint32_t*>(cv.take((size_t)(kDsTop + 2) * 4));
  auto* block_off = static_cast<uint32_t*>(cv.take((size_t)(kDsTop + 2) * 4));
  auto* block_cursor = static_cast<uint32_t*>(cv.take((size_t)(kDsTop + 2) * 4));
  SegBuffers b;
  b.ids = static_cast<int32_t*>(cv.take((size_t)p.nb * 4));
  b.ctrl = static_cast<uint32_t*>(cv.take(kSegCtrlBytes));
  b.blockhist = static_cast<uint32_t*>(cv.take(kSegHistBytes));
  b.quiet = true;
  auto* sample_tmp = static_cast<K*>(cv.take((size_t)p.s * sizeof(K)));
  if (!sample_tmp) return hipErrorInvalidValue;

  // sample and splitters
  const unsigned g = ds_grid(c, n);
  hipLaunchKernelGGL(ds_sample_kernel<K>, dim3(ds_grid(c, p.s)), dim3(kDsThreads), 0, s, keys, n, sample, p.s,
                     (uint64_t)depth * 0x632BE59BD9B4E019ull + (uint64_t)n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = ds_sort<K, 0>(c, sample, nullptr, p.s, sample_tmp, nullptr, cv.p, ws_end, map, s, depth + 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ds_splitter_kernel<K>, dim3(ds_grid(c, p.nspl)), dim3(kDsThreads), 0, s, sample, spl, p.nspl,
                     map);

  // Two-pass partition: the buckets end in keys/vals, sorted there; the
  // single-pass one leaves them in the temporary buffer.
  const int nt = (p.nspl + kDsBlock - 1) / kDsBlock;
  const bool two_pass = nt > kDsTwoPassBlocks;
  K* bk = two_pass ? keys : tmp_keys;  // where the buckets are sorted
  Pay<V>* bv = two_pass ? vals : tmp_vals;
  K* ok = two_pass ? tmp_keys : keys;  // the other buffer: temporary of the recursion
  Pay<V>* ov = two_pass ? tmp_vals : vals;
  e = hipMemsetAsync(nbig, 0, 4, s);
  if (e != hipSuccess) return e;
  if (two_pass) {
    e = hipMemsetAsync(block_count, 0, (size_t)(nt + 1) * 4, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ds_block_count_kernel<K>, dim3(g), dim3(kDsThreads), 0, s, keys, n, spl, p.nspl, block_count,
                       map);
    hipLaunchKernelGGL(ds_block_scan_kernel, dim3(1), dim3(1024), 0, s, block_count, nt + 1, block_off, block_cursor);
    hipLaunchKernelGGL((ds_block_scatter_kernel<K, V>), dim3(g), dim3(kDsThreads), 0, s, keys, vals, n, spl, p.nspl,
                       block_cursor, tmp_keys, tmp_vals, map);
    hipLaunchKernelGGL((ds_block_bucket_kernel<K, V>), dim3(nt + 1), dim3(kDsThreads), 0, s, tmp_keys, tmp_vals, spl,
                       p.nspl, block_off, keys, vals, offsets, p.nb, big, nbig, map);
  } else {
    // count, scan, scatter into the temporary buffer
    e = hipMemsetAsync(counts, 0, (size_t)(p.nb + 1) * 4, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ds_count_kernel<K>, dim3(g), dim3(kDsThreads), 0, s, keys, n, spl, p.nspl, counts, map);
    hipLaunchKernelGGL(ds_scan_kernel, dim3(1), dim3(1024), 0, s, counts, p.nb, offsets, cursors, big, nbig);
    hipLaunchKernelGGL((ds_scatter_kernel<K, V>), dim3(g), dim3(kDsThreads), 0, s, keys, vals, n, spl, p.nspl,
                       cursors, tmp_keys, tmp_vals, map);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;

  // the buckets of at most 4096 keys: one segmented sort (larger ones are skipped)
  if (ds_segmented<K>(c, b, bk, bv, V, offsets, p.nb, map, s) != 0) return hipErrorUnknown;

  // range buckets above 4096 keys: the same sort, with the other buffer (now free) as temporary
  uint32_t nb_host = 0;
  e = hipMemcpyAsync(&nb_host, nbig, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (nb_host > 0) {
    std::vector<uint32_t> bigs(nb_host);
    std::vector<int32_t> offs(p.nb + 1);
    e = hipMemcpyAsync(bigs.data(), big, nb_host * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(offs.data(), offsets, (size_t)(p.nb + 1) * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (uint32_t bi : bigs) {
      const int64_t lo = offs[bi], m = (int64_t)offs[bi + 1] - offs[bi];
      e = ds_sort<K, V>(c, bk + lo, V ? bv + lo : nullptr, m, ok + lo, V ? ov + lo : nullptr, ws, ws_end, map, s,
                        depth + 1);
      if (e != hipSuccess) return e;
    }
  }
  if (!two_pass)
    hipLaunchKernelGGL((ds_copy_kernel<K, V>), dim3(g), dim3(kDsThreads), 0, s, keys, vals, tmp_keys, tmp_vals, n);
  return hipGetLastError();
}

size_t devsort_workspace_bytes(int64_t n, int key_bytes, int val_bytes) {
  const size_t temp = n > kDsBaseN ? ds_align((size_t)n * key_bytes) + ds_align((size_t)n * val_bytes) : 0;
  return temp + ds_level_bytes(n, (size_t)key_bytes) + 256;  // + 256: room to align the base
}

template <class K>
static hipError_t devsort_any(K* keys, void* vals, int vb, int64_t n, void* ws, size_t ws_bytes, KeyMap<K> map,
                              hipStream_t s) {
  hipError_t err = hipSuccess;
  DeviceCtx* c = device_ctx(&err);
  if (!c) return err;
  auto* base = static_cast<unsigned char*>(ws);
  const uintptr_t mis = reinterpret_cast<uintptr_t>(base) & 255;
  if (mis) {  // the carve keeps 256-byte alignment
    if (ws_bytes < 256 - mis) return hipErrorInvalidValue;
    ws_bytes -= 256 - mis;
    base += 256 - mis;
  }
  unsigned char* end = base + ws_bytes;
  const size_t tk = ds_align((size_t)n * sizeof(K));
  const size_t tv = ds_align((size_t)n * (size_t)vb);
  if (n > kDsBaseN && ws_bytes < tk + tv) return hipErrorInvalidValue;
  K* tmp_keys = n > kDsBaseN ? reinterpret_cast<K*>(base) : nullptr;
  unsigned char* rest = n > kDsBaseN ? base + tk + tv : base;
  if (vb == 8) {
    if constexpr (sizeof(K) == 8)
      return ds_sort<K, 8>(c, keys, static_cast<uint64_t*>(vals), n, tmp_keys,
                           reinterpret_cast<uint64_t*>(base + tk), rest, end, map, s, 0);
    return hipErrorInvalidValue;
  }
  if (vb == 4)
    return ds_sort<K, 4>(c, keys, static_cast<uint32_t*>(vals), n, tmp_keys, reinterpret_cast<uint32_t*>(base + tk),
                         rest, end, map, s, 0);
  return ds_sort<K, 0>(c, keys, nullptr, n, tmp_keys, nullptr, rest, end, map, s, 0);
}

hipError_t devsort_u32(uint32_t* keys, void* vals, int vb, int64_t n, void* ws, size_t ws_bytes,
                       KeyMap<uint32_t> map, hipStream_t s) {
  return devsort_any<uint32_t>(keys, vals, vb, n, ws, ws_bytes, map, s);
}
hipError_t devsort_u64(uint64_t* keys, void* vals, int vb, int64_t n, void* ws, size_t ws_bytes,
                       KeyMap<uint64_t> map, hipStream_t s) {
  return devsort_any<uint64_t>(keys, vals, vb, n, ws, ws_bytes, map, s);
}

}  // namespace ss
