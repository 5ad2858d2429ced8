// Entry points of the segmented path for 32- and 64-bit keys: dispatch to the
// instantiation of the current network family and payload width (the kernels
// of each combination are compiled in their own unit; see segmented.hpp).
#include "segmented.hpp"

namespace ss {

int segmented_u32(DeviceCtx* c, uint32_t* keys, void* vals, int vbytes, const int32_t* offsets, int32_t nseg,
                  KeyMap<uint32_t> flip, int mode, hipStream_t s) {
  return segmented_any<uint32_t>(c, keys, vals, vbytes, offsets, nseg, flip, mode, s);
}

int segmented_u64(DeviceCtx* c, uint64_t* keys, void* vals, int vbytes, const int32_t* offsets, int32_t nseg,
                  KeyMap<uint64_t> flip, int mode, hipStream_t s) {
  return segmented_any<uint64_t>(c, keys, vals, vbytes, offsets, nseg, flip, mode, s);
}

int segmented_direct_u32(DeviceCtx* c, const SegBuffers& b, uint32_t* keys, void* vals, int vbytes,
                         const int32_t* offsets, int32_t nseg, KeyMap<uint32_t> flip, hipStream_t s) {
  return segmented_direct_any<uint32_t>(c, b, keys, vals, vbytes, offsets, nseg, flip, s);
}

int segmented_direct_u64(DeviceCtx* c, const SegBuffers& b, uint64_t* keys, void* vals, int vbytes,
                         const int32_t* offsets, int32_t nseg, KeyMap<uint64_t> flip, hipStream_t s) {
  return segmented_direct_any<uint64_t>(c, b, keys, vals, vbytes, offsets, nseg, flip, s);
}

}  // namespace ss
