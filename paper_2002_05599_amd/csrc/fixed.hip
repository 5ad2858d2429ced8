// Comparator-network sort of many arrays of N = 2..16 keys (paper, Section 2).
//
// One thread sorts one array held in N registers (Section 2.2: straight-line
// conditional swaps with no branches; here each swap is v_min/v_max for 32-bit
// keys).  Arrays sit back to back in HBM (the ArrayInRow layout of
// Section 4.1), so a thread's own keys are N*sizeof(K) contiguous bytes and a
// direct per-thread load would touch a different 16-byte piece of many cache
// lines per instruction.  Instead a work-group stages its tile of arrays
// through LDS (256 threads and arrays; per n, as tuned, 128 threads and
// arrays, or 512 or 1024 threads moving a tile of 256 arrays):
//
//   HBM --(16-byte coalesced loads, consecutive lanes -> consecutive bytes)--> VGPRs
//       --(LDS write in a conflict-avoiding layout)--> LDS
//       --(each thread reads its own row)--> N VGPRs --network--> LDS --> HBM
//
// LDS layouts (chosen at compile time from N and the key size E):
//   * vector layout, when N*E is a multiple of 16: each array is C = N*E/16
//     chunks of 16 bytes; chunk k of array a is stored in slot a*C + rot(a, k)
//     with a per-array rotation, so the 16-byte reads of 8 neighbouring
//     threads (one LDS pass) fall in distinct bank groups;
//   * element layout otherwise: array a occupies elements [a*P, a*P+N) with
//     an odd pitch P (N or N+1), so a wave's per-thread element reads hit
//     distinct banks.
// The last, partial tile (count not a multiple of the tile) takes element-wise
// global accesses guarded by bounds.  A stride other than N, or a base pointer
// that is not 16-byte aligned, uses the direct per-thread kernel instead.
#include "common.hpp"
#include "internal.hpp"

namespace ss {

constexpr int kTileThreads = 256;

// Native 16-byte vector (the HIP uint4 struct is not accepted by the
// non-temporal builtins).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Tile of TA = A * TT arrays (A arrays per thread, TT threads).
template <int N, class K, int A = 1, int TT = kTileThreads> struct TileLayout {
  static constexpr int TA = A * TT;
  static constexpr int E = (int)sizeof(K);
  static constexpr bool kVec = (N * E) % 16 == 0;
  static constexpr int C = kVec ? N * E / 16 : 1;   // 16-byte chunks per array
  static constexpr int P = (N % 2) ? N : N + 1;    // element pitch (element layout)
  static constexpr int kBytes = kVec ? TA * N * E : TA * P * E;
  static constexpr int kPerChunk = 16 / E;         // keys per 16-byte chunk
  // odd N: the element layout (pitch N) is the tile's own byte order, so
  // 16-byte chunks move between HBM and LDS whole
  static constexpr bool kLinear = !kVec && P == N;
  // Rotation step: threads a and a' whose rows start in the same bank group
  // within one 8-thread pass get different rotations.
  static constexpr int kRotShift = (C == 2) ? 2 : (C == 4) ? 1 : (C == 6) ? 2 : 0;

  __device__ __forceinline__ static int chunk_slot(int a, int k) {
    if constexpr (C % 2 == 1) {
      return a * C + k;
    } else {
      int r = (a >> kRotShift) % C;
      int kk = k + r;
      kk = kk >= C ? kk - C : kk;
      return a * C + kk;
    }
  }
  // Byte offset in LDS of key j of array a.
  __device__ __forceinline__ static int elem_offset(int a, int j) {
    if constexpr (kVec) {
      return chunk_slot(a, j / kPerChunk) * 16 + (j % kPerChunk) * E;
    } else {
      return (a * P + j) * E;
    }
  }
};

// Arrays per thread that a tile may use: the tile's LDS stays within 32 KiB
// (so that the work-groups of one CU keep enough waves to hide HBM latency).
template <int N, class K, int A>
constexpr bool tile_fits() { return TileLayout<N, K, A>::kBytes <= 32768; }

template <class K> __device__ __forceinline__ K lds_ld(const unsigned char* p) {
  return *reinterpret_cast<const K*>(p);
}
template <class K> __device__ __forceinline__ void lds_st(unsigned char* p, K v) {
  *reinterpret_cast<K*>(p) = v;
}

// One tile of A * TS arrays moved by TT threads (TT = TS = 256; 128 for a
// one-array-per-thread tile of half the LDS; TT = 512 or 1024 over TS = 256
// arrays, where every thread moves a half or a quarter as many chunks and the
// first 256 sort).
template <int F, int N, class K, int A, int TT, int TS = TT>
__device__ __forceinline__ void tile_sort(K* __restrict__ keys, int64_t count, KeyMap<K> flip) {
  using L = TileLayout<N, K, A, TS>;
  constexpr int TA = L::TA;
  __shared__ __attribute__((aligned(16))) unsigned char lds[L::kBytes];
  constexpr int kChunks = TA * N * L::E / 16;  // 16-byte chunks in a full tile
  constexpr int kIters = (kChunks + TT - 1) / TT;
  constexpr bool kExact = (kChunks % TT) == 0;

  const int t = threadIdx.x;
  const int64_t first = (int64_t)blockIdx.x * TA;
  const int64_t left = count - first;
  const int valid = left < TA ? (int)left : TA;
  K* gk = keys + first * N;
  const bool full = valid == TA;

  if (full) {
    const u32x4* g4 = reinterpret_cast<const u32x4*>(gk);
    u32x4 buf[kIters];
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
      int g = t + i * TT;
      if (kExact || g < kChunks) buf[i] = __builtin_nontemporal_load(g4 + g);
    }
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
      int g = t + i * TT;
      if (kExact || g < kChunks) {
        if constexpr (L::kVec) {
          int a = g / L::C, k = g - (g / L::C) * L::C;
          *reinterpret_cast<u32x4*>(lds + L::chunk_slot(a, k) * 16) = buf[i];
        } else if constexpr (L::kLinear) {
          *reinterpret_cast<u32x4*>(lds + g * 16) = buf[i];
        } else {
          K parts[L::kPerChunk];
          __builtin_memcpy(parts, &buf[i], 16);
#pragma unroll
          for (int q = 0; q < L::kPerChunk; ++q) {
            int e = g * L::kPerChunk + q;
            int a = e / N, j = e - (e / N) * N;
            lds_st<K>(lds + L::elem_offset(a, j), parts[q]);
          }
        }
      }
    }
  } else {
    const int nelem = valid * N;
    for (int e = t; e < nelem; e += TT) {
      int a = e / N, j = e - (e / N) * N;
      lds_st<K>(lds + L::elem_offset(a, j), gk[e]);
    }
  }
  __syncthreads();

#pragma unroll
  for (int q = 0; q < A; ++q) {
    const int a = t + q * TS;  // this thread's q-th array of the tile (none for t >= TS)
    if (a < valid) {
      K r[N];
      if constexpr (L::kVec) {
#pragma unroll
        for (int k = 0; k < L::C; ++k) {
          u32x4 v = *reinterpret_cast<const u32x4*>(lds + L::chunk_slot(a, k) * 16);
          __builtin_memcpy(&r[k * L::kPerChunk], &v, 16);
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = lds_ld<K>(lds + L::elem_offset(a, j));
      }
      flip.enc_all(r);
      net_sort<F, N>(r);
      flip.dec_all(r);
      if constexpr (L::kVec) {
#pragma unroll
        for (int k = 0; k < L::C; ++k) {
          u32x4 v;
          __builtin_memcpy(&v, &r[k * L::kPerChunk], 16);
          *reinterpret_cast<u32x4*>(lds + L::chunk_slot(a, k) * 16) = v;
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) lds_st<K>(lds + L::elem_offset(a, j), r[j]);
      }
    }
  }
  __syncthreads();

  if (full) {
    u32x4* g4 = reinterpret_cast<u32x4*>(gk);
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
      int g = t + i * TT;
      if (kExact || g < kChunks) {
        u32x4 v;
        if constexpr (L::kVec) {
          int a = g / L::C, k = g - (g / L::C) * L::C;
          v = *reinterpret_cast<const u32x4*>(lds + L::chunk_slot(a, k) * 16);
        } else if constexpr (L::kLinear) {
          v = *reinterpret_cast<const u32x4*>(lds + g * 16);
        } else {
          K parts[L::kPerChunk];
#pragma unroll
          for (int q = 0; q < L::kPerChunk; ++q) {
            int e = g * L::kPerChunk + q;
            int a = e / N, j = e - (e / N) * N;
            parts[q] = lds_ld<K>(lds + L::elem_offset(a, j));
          }
          __builtin_memcpy(&v, parts, 16);
        }
        __builtin_nontemporal_store(v, g4 + g);
      }
    }
  } else {
    const int nelem = valid * N;
    for (int e = t; e < nelem; e += TT) {
      int a = e / N, j = e - (e / N) * N;
      gk[e] = lds_ld<K>(lds + L::elem_offset(a, j));
    }
  }
}

template <int F, int N, class K, int A>
__global__ void __launch_bounds__(kTileThreads)
fixed_tile_kernel(K* __restrict__ keys, int64_t count, KeyMap<K> flip) {
  tile_sort<F, N, K, A, kTileThreads>(keys, count, flip);
}

// The one-array-per-thread tile with 128 threads.  A network tile asks for at
// least kTileMinWaves waves per SIMD, so that the compiler does not trade
// occupancy for registers (it would hoist every chunk load of a tile of 64-bit
// keys into registers otherwise); insertion sort keeps the default bound,
// which avoids spills.
constexpr int kHalfTileThreads = 128;
constexpr int kTileMinWaves = 4;
template <int F, int N, class K>
__global__ void __launch_bounds__(kHalfTileThreads, F != kFamilyInsertion ? kTileMinWaves : 1)
fixed_half_tile_kernel(K* __restrict__ keys, int64_t count, KeyMap<K> flip) {
  tile_sort<F, N, K, 1, kHalfTileThreads>(keys, count, flip);
}

// The one-array-per-thread tile of 256 arrays moved by 512 threads: each
// thread loads and stores half as many 16-byte chunks, the first 256 threads
// sort.
constexpr int kWideTileThreads = 512;
template <int F, int N, class K>
__global__ void __launch_bounds__(kWideTileThreads)
fixed_wide_tile_kernel(K* __restrict__ keys, int64_t count, KeyMap<K> flip) {
  tile_sort<F, N, K, 1, kWideTileThreads, kTileThreads>(keys, count, flip);
}

// The same with 1024 threads (a quarter of the chunks per thread).
constexpr int kWiderTileThreads = 1024;
template <int F, int N, class K>
__global__ void __launch_bounds__(kWiderTileThreads)
fixed_wider_tile_kernel(K* __restrict__ keys, int64_t count, KeyMap<K> flip) {
  tile_sort<F, N, K, 1, kWiderTileThreads, kTileThreads>(keys, count, flip);
}

// Arrays of 8 bytes (uint32 n = 2): a 16-byte chunk holds two whole arrays,
// so every thread loads its chunks straight from HBM (consecutive lanes,
// consecutive chunks: fully coalesced), sorts them in registers and stores
// them back; no LDS staging.  (For 16-byte arrays the staged tile measured
// faster.)  One chunk per thread: on 2^24 arrays 1, 2, 4 and 8 chunks per
// thread measured 0.77, 0.755, 0.71-0.72 and 0.70 of 8 TB/s.
constexpr int kVecChunks = 1;  // chunks per thread
template <int F, int N, class K>
__global__ void __launch_bounds__(kTileThreads)
fixed_vec_kernel(K* __restrict__ keys, int64_t chunks, KeyMap<K> flip) {
  constexpr int kArr = 16 / (N * (int)sizeof(K));  // arrays per chunk
  static_assert(kArr * N * (int)sizeof(K) == 16, "one or two whole arrays per chunk");
  const int64_t base = (int64_t)blockIdx.x * (kTileThreads * kVecChunks) + threadIdx.x;
  u32x4* g4 = reinterpret_cast<u32x4*>(keys);
  u32x4 buf[kVecChunks];
#pragma unroll
  for (int i = 0; i < kVecChunks; ++i) {
    const int64_t c = base + (int64_t)i * kTileThreads;
    if (c < chunks) buf[i] = __builtin_nontemporal_load(g4 + c);
  }
#pragma unroll
  for (int i = 0; i < kVecChunks; ++i) {
    const int64_t c = base + (int64_t)i * kTileThreads;
    if (c < chunks) {
      K r[kArr * N];
      __builtin_memcpy(r, &buf[i], 16);
#pragma unroll
      for (int q = 0; q < kArr; ++q) {
        K a[N];
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = r[q * N + j];
        flip.enc_all(a);
        net_sort<F, N>(a);
        flip.dec_all(a);
#pragma unroll
        for (int j = 0; j < N; ++j) r[q * N + j] = a[j];
      }
      u32x4 v;
      __builtin_memcpy(&v, r, 16);
      __builtin_nontemporal_store(v, g4 + c);
    }
  }
}

// One thread per array, direct global accesses: any stride, any alignment.
template <int F, int N, class K>
__global__ void __launch_bounds__(kTileThreads)
fixed_direct_kernel(K* __restrict__ keys, int64_t count, int64_t stride, KeyMap<K> flip) {
  const int64_t a = (int64_t)blockIdx.x * kTileThreads + threadIdx.x;
  if (a >= count) return;
  K* p = keys + a * stride;
  K r[N];
#pragma unroll
  for (int j = 0; j < N; ++j) r[j] = flip.enc(p[j]);
  net_sort<F, N>(r);
#pragma unroll
  for (int j = 0; j < N; ++j) p[j] = flip.dec(r[j]);
}

template <int F, int N, class K, int A, int TT = kTileThreads>
static hipError_t launch_tile(K* keys, int64_t count, KeyMap<K> flip, hipStream_t s) {
  constexpr int64_t TA = (int64_t)A * (TT > kTileThreads ? kTileThreads : TT);  // arrays per work-group
  const int64_t blocks = (count + TA - 1) / TA;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  if constexpr (TT == kHalfTileThreads) {
    static_assert(A == 1, "the 128-thread tile holds one array per thread");
    hipLaunchKernelGGL((fixed_half_tile_kernel<F, N, K>), dim3((unsigned)blocks), dim3(TT), 0, s, keys, count, flip);
  } else if constexpr (TT == kWideTileThreads) {
    static_assert(A == 1, "the 512-thread tile holds 256 arrays");
    hipLaunchKernelGGL((fixed_wide_tile_kernel<F, N, K>), dim3((unsigned)blocks), dim3(TT), 0, s, keys, count, flip);
  } else if constexpr (TT == kWiderTileThreads) {
    static_assert(A == 1, "the 1024-thread tile holds 256 arrays");
    hipLaunchKernelGGL((fixed_wider_tile_kernel<F, N, K>), dim3((unsigned)blocks), dim3(TT), 0, s, keys, count, flip);
  } else {
    hipLaunchKernelGGL((fixed_tile_kernel<F, N, K, A>), dim3((unsigned)blocks), dim3(TT), 0, s, keys, count, flip);
  }
  return hipGetLastError();
}

template <int F, int N, class K>
static hipError_t launch_fixed_n(K* keys, int64_t count, int64_t stride, KeyMap<K> flip, int apt, bool half,
                                 bool wide, bool wider, hipStream_t s) {
  const int64_t blocks = (count + kTileThreads - 1) / kTileThreads;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  const bool tiled = stride == N && (reinterpret_cast<uintptr_t>(keys) % 16) == 0;
  if constexpr (N * sizeof(K) == 8) {
    if (tiled) {
      constexpr int64_t kArr = 16 / (N * sizeof(K));
      const int64_t chunks = count / kArr;
      const int64_t per = (int64_t)kTileThreads * kVecChunks;
      const int64_t vblocks = (chunks + per - 1) / per;
      if (vblocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
      if (chunks > 0)
        hipLaunchKernelGGL((fixed_vec_kernel<F, N, K>), dim3((unsigned)vblocks), dim3(kTileThreads), 0, s, keys,
                           chunks, flip);
      if (chunks * kArr < count)  // an odd count of two-array chunks: the last array alone
        hipLaunchKernelGGL((fixed_direct_kernel<F, N, K>), dim3(1), dim3(kTileThreads), 0, s,
                           keys + chunks * kArr * N, (int64_t)1, (int64_t)N, flip);
      return hipGetLastError();
    }
  }
  if (tiled) {
    // arrays per thread: the tuned value, or the largest smaller one whose tile fits
    if constexpr (tile_fits<N, K, 4>()) {
      if (apt >= 4) return launch_tile<F, N, K, 4>(keys, count, flip, s);
    }
    if constexpr (tile_fits<N, K, 2>()) {
      if (apt >= 2) return launch_tile<F, N, K, 2>(keys, count, flip, s);
    }
    // the wide forms serve the networks (insertion sort spills under their register budget)
    if constexpr (F != kFamilyInsertion) {
      if (wider) return launch_tile<F, N, K, 1, kWiderTileThreads>(keys, count, flip, s);
      if (wide) return launch_tile<F, N, K, 1, kWideTileThreads>(keys, count, flip, s);
    }
    if (half) return launch_tile<F, N, K, 1, kHalfTileThreads>(keys, count, flip, s);
    return launch_tile<F, N, K, 1>(keys, count, flip, s);
  } else {
    hipLaunchKernelGGL((fixed_direct_kernel<F, N, K>), dim3((unsigned)blocks), dim3(kTileThreads), 0, s,
                       keys, count, stride, flip);
  }
  return hipGetLastError();
}

template <int F, class K>
static hipError_t launch_fixed_f(K* keys, int n, int64_t count, int64_t stride, KeyMap<K> flip, hipStream_t s) {
  const Tuning t = tuning(sizeof(K));
  const int apt = t.fixed_apt;
  const bool half = ((t.fixed_half >> n) & 1) != 0;
  const bool wide = ((t.fixed_wide >> n) & 1) != 0;
  const bool wider = ((t.fixed_wider >> n) & 1) != 0;
  switch (n) {
    case 2: return launch_fixed_n<F, 2>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 3: return launch_fixed_n<F, 3>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 4: return launch_fixed_n<F, 4>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 5: return launch_fixed_n<F, 5>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 6: return launch_fixed_n<F, 6>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 7: return launch_fixed_n<F, 7>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 8: return launch_fixed_n<F, 8>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 9: return launch_fixed_n<F, 9>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 10: return launch_fixed_n<F, 10>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 11: return launch_fixed_n<F, 11>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 12: return launch_fixed_n<F, 12>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 13: return launch_fixed_n<F, 13>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 14: return launch_fixed_n<F, 14>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 15: return launch_fixed_n<F, 15>(keys, count, stride, flip, apt, half, wide, wider, s);
    case 16: return launch_fixed_n<F, 16>(keys, count, stride, flip, apt, half, wide, wider, s);
    default: return hipErrorInvalidValue;
  }
}

// Streaming copy with the tile kernels' access pattern: each thread moves
// 16-byte chunks with nontemporal loads and stores, consecutive lanes on
// consecutive chunks, kCopyIters chunks per thread (on 1 GiB, 1, 2 and 4
// chunks per thread measured 0.81, 0.76 and 0.78 of 8 TB/s).
constexpr int kCopyIters = 1;
__global__ void __launch_bounds__(kTileThreads)
stream_copy_kernel(u32x4* __restrict__ dst, const u32x4* __restrict__ src, int64_t chunks) {
  const int64_t base = (int64_t)blockIdx.x * (kTileThreads * kCopyIters) + threadIdx.x;
  u32x4 buf[kCopyIters];
#pragma unroll
  for (int i = 0; i < kCopyIters; ++i) {
    const int64_t c = base + (int64_t)i * kTileThreads;
    if (c < chunks) buf[i] = __builtin_nontemporal_load(src + c);
  }
#pragma unroll
  for (int i = 0; i < kCopyIters; ++i) {
    const int64_t c = base + (int64_t)i * kTileThreads;
    if (c < chunks) __builtin_nontemporal_store(buf[i], dst + c);
  }
}

hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
  const int64_t chunks = bytes / 16;
  const int64_t per_block = (int64_t)kTileThreads * kCopyIters;
  const int64_t blocks = (chunks + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFFLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kTileThreads), 0, s,
                     static_cast<u32x4*>(dst), static_cast<const u32x4*>(src), chunks);
  return hipGetLastError();
}

hipError_t launch_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                            hipStream_t s) {
  switch (tuning(sizeof(*keys)).family) {
    case 1: return launch_fixed_f<1>(keys, n, count, stride, flip, s);
    case kFamilyInsertion: return launch_fixed_f<kFamilyInsertion>(keys, n, count, stride, flip, s);
    default: return launch_fixed_f<0>(keys, n, count, stride, flip, s);
  }
}
hipError_t launch_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                            hipStream_t s) {
  switch (tuning(sizeof(*keys)).family) {
    case 1: return launch_fixed_f<1>(keys, n, count, stride, flip, s);
    case kFamilyInsertion: return launch_fixed_f<kFamilyInsertion>(keys, n, count, stride, flip, s);
    default: return launch_fixed_f<0>(keys, n, count, stride, flip, s);
  }
}

}  // namespace ss
