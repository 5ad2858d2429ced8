#include "internal.hpp"
namespace ss {
int segmented_u32(DeviceCtx*, uint32_t*, uint32_t*, const int32_t*, int32_t, uint32_t, int, hipStream_t) { return -4; }
int segmented_u64(DeviceCtx*, uint64_t*, uint32_t*, const int32_t*, int32_t, uint64_t, int, hipStream_t) { return -4; }
}
