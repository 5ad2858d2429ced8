#include "internal.hpp"
namespace ss {
hipError_t launch_rss_fixed_u32(uint32_t*, int, int64_t, int64_t, uint32_t, int*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_rss_fixed_u64(uint64_t*, int, int64_t, int64_t, uint64_t, int*, hipStream_t) { return hipErrorNotSupported; }
int segmented_u32(DeviceCtx*, uint32_t*, uint32_t*, const int32_t*, int32_t, uint32_t, int, hipStream_t) { return -4; }
int segmented_u64(DeviceCtx*, uint64_t*, uint32_t*, const int32_t*, int32_t, uint64_t, int, hipStream_t) { return -4; }
}
