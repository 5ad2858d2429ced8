// Host-side interfaces between the C ABI (capi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "keymap.hpp"

namespace ss {

// Variant choices, set by the autotuner through ss_set_tuning_value.
struct Tuning {
  int family = 0;        // n <= 16: 0 fewest-comparator networks, 1 Bose-Nelson, 2 insertion sort
  int rss_k[3] = {16, 32, 64};  // level-0 bucket count for 17..64, 65..128, 129..256 keys
  int persist_occ = 0;   // work-groups per CU for the persistent grid (0 = occupancy limit)
  int rss_rounds = 16;    // rounds of groups per RSS tile in the segmented kernels
  int interleave = 1;    // persistent kernel alternates RSS and network tiles
  int persist_split = 1;  // 1: one persistent kernel per kind (networks, each RSS class); 0: one for all
  int net_mix = 0;        // 1: persistent forms sort 2..16-key segments in batch order, mixed sizes
  int rss_level_cap = 8;  // RSS levels before the rank-counting fallback finishes a pending bucket
  int large_sort = 0;     // 17..256 keys: 0 Register Sample Sort, 1 insertion sort (the IS+SN hybrid)
  int rss_bound_small = 64;  // largest segment sorted by a 16-lane RSS group (16..64)
  int rss_bound_mid = 128;   // largest segment sorted by a 32-lane RSS group (bound_small..128)
  int rss_oversample = 3;    // oversampling a of the RSS levels with 4 buckets (1..4)
  int fixed_apt = 1;         // arrays per thread of the fixed-layout network kernels (1, 2, 4)
  int fixed_half = 0;        // bit n: arrays of n keys use the 128-thread one-array-per-thread tile
  int fixed_wide = 0;        // bit n: ... the 512-thread tile of 256 arrays (over fixed_half)
  int fixed_wider = 0;       // bit n: ... the 1024-thread tile of 256 arrays (over both)
  int rss_bound_tiny = 16;   // largest segment sorted by an 8-lane RSS group (16 = none, ..32)
  int rss_finish = 0;        // RSS buckets finished by 0 networks, 1 rank counting
};
// A consistent copy of the current settings for keys of key_bytes (4 or 8)
// bytes: the variant choices are kept per key width.
Tuning tuning(int key_bytes);

// Fixed layout, n = 2..16 (networks).  flip = the key type's order-preserving map.
hipError_t launch_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                            hipStream_t s);
hipError_t launch_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                            hipStream_t s);

// Fixed layout, n = 17..256 (Register Sample Sort).
hipError_t launch_rss_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                                int* status, hipStream_t s);
hipError_t launch_rss_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                                int* status, hipStream_t s);

// Fixed layout, n = 257..4096 (runs sorted by RSS, merged in LDS).
hipError_t launch_large_fixed_u32(uint32_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint32_t> flip,
                                  hipStream_t s);
hipError_t launch_large_fixed_u64(uint64_t* keys, int n, int64_t count, int64_t stride, KeyMap<uint64_t> flip,
                                  hipStream_t s);

// One large array (n < 2^31) sorted with the small sorters as base case
// (devsort.hip); vb = payload bytes (0, 4, 8); synchronises s.
size_t devsort_workspace_bytes(int64_t n, int key_bytes, int val_bytes);
hipError_t devsort_u32(uint32_t* keys, void* vals, int vb, int64_t n, void* ws, size_t ws_bytes,
                       KeyMap<uint32_t> map, hipStream_t s);
hipError_t devsort_u64(uint64_t* keys, void* vals, int vb, int64_t n, void* ws, size_t ws_bytes,
                       KeyMap<uint64_t> map, hipStream_t s);

// Streaming device-to-device copy of `bytes` (the read-once / write-once
// ceiling the sorting kernels are measured against).
hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

// Per-device context: status word, device properties and working memory
// for the segmented path (grown on demand, freed at process exit).
struct SegRegistry;  // per-stream working memory of the segmented path
struct DeviceCtx {
  int device = -1;
  int num_cus = 0;
  int* status = nullptr;       // device int32 status word
  SegRegistry* seg = nullptr;  // segmented-path workspaces, one per stream
  void* scratch = nullptr;     // this device's address of the fixed no-allocation scratch array
};

// Device working memory of one segmented call: the segment-id list grouped by
// size class, the control block (class counts, class starts, claim counters)
// and the per-block class histogram of the binning.
struct SegBuffers {
  int32_t* ids = nullptr;
  uint32_t* ctrl = nullptr;    // kSegCtrlBytes
  uint32_t* blockhist = nullptr;  // kSegHistBytes
  bool quiet = false;  // skip segments above 4096 keys without flagging them in the status word
};
// Sizes of the binning's control block and per-block class histogram (1024
// blocks x 20 size classes).
constexpr size_t kSegCtrlBytes = 8192;
constexpr size_t kSegHistBytes = 1024 * 20 * 4;

// Largest batch of the no-allocation segmented entry point (its segment-id
// list lives in the fixed scratch array).
constexpr int32_t kNoAllocMaxSeg = 1 << 24;
// The scratch array carved into SegBuffers for `nseg` <= kNoAllocMaxSeg
// segments; the device address is looked up once per device (hipGetSymbolAddress).
hipError_t noalloc_buffers(DeviceCtx* c, SegBuffers* out);
// Context of the current device, created on first use; nullptr on failure
// with *err set to a HIP error.
DeviceCtx* device_ctx(hipError_t* err);

// Segmented (CSR) sorting; returns an ss_status code.  vals: NULL or a
// payload of vbytes = 4 (uint32) or 8 (uint64, 64-bit keys only) per key.
// mode: 0 persistent kernel from a cached graph, 1 persistent kernel launched
// directly, 2 one plain launch per size class.
int segmented_u32(DeviceCtx* c, uint32_t* keys, void* vals, int vbytes, const int32_t* offsets, int32_t nseg,
                  KeyMap<uint32_t> flip, int mode, hipStream_t s);
int segmented_u64(DeviceCtx* c, uint64_t* keys, void* vals, int vbytes, const int32_t* offsets, int32_t nseg,
                  KeyMap<uint64_t> flip, int mode, hipStream_t s);
// The same sorts with the persistent kernels launched directly on the given
// buffers (no graph, no working-memory allocation): the no-allocation path.
int segmented_direct_u32(DeviceCtx* c, const SegBuffers& b, uint32_t* keys, void* vals, int vbytes,
                         const int32_t* offsets, int32_t nseg, KeyMap<uint32_t> flip, hipStream_t s);
int segmented_direct_u64(DeviceCtx* c, const SegBuffers& b, uint64_t* keys, void* vals, int vbytes,
                         const int32_t* offsets, int32_t nseg, KeyMap<uint64_t> flip, hipStream_t s);

}  // namespace ss
