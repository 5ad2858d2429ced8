// Binning kernels and working memory of the segmented path (see segmented.hpp).
#include "segmented.hpp"

namespace ss {

__global__ void __launch_bounds__(kBinThreads)
seg_count_kernel(const int32_t* __restrict__ offsets, int32_t nseg, uint32_t* __restrict__ blockhist,
                 int* status, int bins) {
  __shared__ uint32_t hist[kClasses];
  if (threadIdx.x < kClasses) hist[threadIdx.x] = 0;
  __syncthreads();
  int bad = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBinChunk; base < nseg; base += (int64_t)gridDim.x * kBinChunk) {
#pragma unroll
    for (int q = 0; q < kBinItems; ++q) {
      const int64_t i = base + q * kBinThreads + threadIdx.x;
      if (i < nseg) {
        const int c = bin_class(offsets[i + 1] - offsets[i], bins);
        if (c >= 0)
          atomicAdd(&hist[c], 1u);
        else if (c < -1)
          bad = c == -2 ? kStatusTooBig : kStatusInval;
      }
    }
  }
  if (bad) report(status, bad);
  __syncthreads();
  if (threadIdx.x < kClasses) blockhist[threadIdx.x * kBinBlocks + blockIdx.x] = hist[threadIdx.x];
}

// One block of 1024 threads: class totals, class starts, per-block bases
// (written over the per-block histogram), tile counter reset.  The histogram
// is laid out [class][block]; one wave scans one class row of kBinBlocks
// values, 16 per lane.
__global__ void __launch_bounds__(1024)
seg_scan_kernel(uint32_t* __restrict__ blockhist, int nblocks, uint32_t* __restrict__ ctrl) {
  constexpr int kPerLane = kBinBlocks / kWave;
  __shared__ uint32_t tot[kClasses];
  const int wave = threadIdx.x / kWave;
  const int lane = lane_id();
  (void)nblocks;
  for (int c = wave; c < kClasses; c += 1024 / kWave) {
    uint32_t* row = blockhist + c * kBinBlocks + lane * kPerLane;
    uint32_t v[kPerLane];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
      v[i] = row[i];
      sum += v[i];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, d);
      if (lane >= d) incl += y;
    }
    uint32_t run = incl - sum;
#pragma unroll
    for (int i = 0; i < kPerLane; ++i) {
      row[i] = run;
      run += v[i];
    }
    if (lane == kWave - 1) tot[c] = incl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t st = 0;
    for (int c = 0; c < kClasses; ++c) {
      ctrl[kCtrlCount + c] = tot[c];
      ctrl[kCtrlStart + c] = st;
      st += tot[c];
    }
    for (int k = 0; k < kKinds * kTileParts; ++k) ctrl[kCtrlTile + k * 32] = 0;
  }
}

__global__ void __launch_bounds__(kBinThreads)
seg_scatter_kernel(const int32_t* __restrict__ offsets, int32_t nseg, const uint32_t* __restrict__ blockbase,
                   const uint32_t* __restrict__ ctrl, int32_t* __restrict__ ids, int bins) {
  __shared__ uint32_t cur[kClasses];
  if (threadIdx.x < kClasses)
    cur[threadIdx.x] = ctrl[kCtrlStart + threadIdx.x] + blockbase[threadIdx.x * kBinBlocks + blockIdx.x];
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * kBinChunk; base < nseg; base += (int64_t)gridDim.x * kBinChunk) {
#pragma unroll
    for (int q = 0; q < kBinItems; ++q) {
      const int64_t i = base + q * kBinThreads + threadIdx.x;
      if (i < nseg) {
        const int c = bin_class(offsets[i + 1] - offsets[i], bins);
        if (c >= 0) ids[atomicAdd(&cur[c], 1u)] = (int32_t)i;
      }
    }
  }
}

// --- fixed scratch of the no-allocation entry point ---------------------------
//
// One array per device, held from code-object load until the process ends:
// the control block, the binning histogram and a segment-id list for up to
// kNoAllocMaxSeg segments (64 MiB + 88 KiB).  Every no-allocation call on a
// device uses the same array, so such calls must not overlap on one device.
// Nothing in it needs clearing between calls: the count kernel writes every
// histogram entry, the scan kernel writes the class counts and starts and
// zeroes the claim counters, the scatter kernel writes the ids it uses.
constexpr size_t kScratchCtrlBytes = 8192;
constexpr size_t kScratchHistBytes = (size_t)kBinBlocks * kClasses * sizeof(uint32_t);
constexpr size_t kScratchBytes = kScratchCtrlBytes + kScratchHistBytes + (size_t)kNoAllocMaxSeg * sizeof(int32_t);
static_assert(kCtrlWords * sizeof(uint32_t) <= kScratchCtrlBytes, "control block must fit its scratch slot");
static_assert(kScratchHistBytes % 256 == 0, "histogram slot keeps the id list 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t noalloc_buffers(DeviceCtx* c, SegBuffers* out) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (!c->scratch) {
    // `scratch` names a host-side stand-in; the device address of this
    // device's copy comes from the runtime (the caller made c's device current).
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    c->scratch = p;
  }
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  out->ctrl = reinterpret_cast<uint32_t*>(base);
  out->blockhist = reinterpret_cast<uint32_t*>(base + kScratchCtrlBytes);
  out->ids = reinterpret_cast<int32_t*>(base + kScratchCtrlBytes + kScratchHistBytes);
  return hipSuccess;
}

struct SegRegistry {
  std::mutex mu;
  std::vector<std::pair<hipStream_t, SegmentedCache*>> list;
};

SegmentedCache* workspace_for(DeviceCtx* c, hipStream_t s) {
  static std::mutex create_mu;
  {
    std::lock_guard<std::mutex> lock(create_mu);
    if (!c->seg) c->seg = new SegRegistry();
  }
  SegRegistry* r = c->seg;
  std::lock_guard<std::mutex> lock(r->mu);
  for (auto& e : r->list)
    if (e.first == s) return e.second;
  SegmentedCache* ws = new SegmentedCache();
  hipError_t e = hipMalloc(&ws->ctrl, kCtrlWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&ws->blockhist, kBinBlocks * kClasses * sizeof(uint32_t));
  if (e == hipSuccess) e = hipHostMalloc(&ws->host_ctrl, kCtrlWords * sizeof(uint32_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (ws->ctrl) (void)hipFree(ws->ctrl);
    if (ws->blockhist) (void)hipFree(ws->blockhist);
    delete ws;
    return nullptr;
  }
  r->list.emplace_back(s, ws);
  return ws;
}

hipError_t ensure_workspace(SegmentedCache* s, int32_t nseg, hipStream_t stream) {
  if (s->ids_cap >= nseg) return hipSuccess;
  // Growing, ordered on the workspace's own stream (the only stream that uses
  // it): the old list is released after the work already queued there, and
  // the new one is ready for the work queued next.  No host or device sync.
  hipError_t e = hipSuccess;
  if (s->ids) e = hipFreeAsync(s->ids, stream);
  s->ids = nullptr;
  s->ids_cap = 0;
  int64_t cap = nseg < 1024 ? 1024 : (int64_t)nseg + nseg / 4;
  if (cap > 0x7FFFFFFF) cap = 0x7FFFFFFF;
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&s->ids), cap * sizeof(int32_t), stream);
  if (e != hipSuccess) {
    s->ids = nullptr;
    return e;
  }
  s->ids_cap = cap;
  return hipSuccess;
}

}  // namespace ss
