// Segmented sort entry for uint32_t keys (kernels instantiated here; see segmented.hpp).
#include "segmented.hpp"

namespace ss {

int segmented_u32(DeviceCtx* c, uint32_t* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg, uint32_t flip,
                  int mode, hipStream_t s) {
  return segmented_any<uint32_t>(c, keys, vals, offsets, nseg, flip, mode, s);
}

int segmented_direct_u32(DeviceCtx* c, const SegBuffers& b, uint32_t* keys, uint32_t* vals, const int32_t* offsets,
                         int32_t nseg, uint32_t flip, hipStream_t s) {
  return segmented_direct_any<uint32_t>(c, b, keys, vals, offsets, nseg, flip, s);
}

}  // namespace ss
