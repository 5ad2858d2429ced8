// C ABI of libsmallsort.so: argument checks, dispatch by size and key type,
// tuning parameters and the per-device status word.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/smallsort.h"
#include "internal.hpp"

namespace ss {

// The process-wide tuning values, one set per key width (index 0: 32-bit
// keys, 1: 64-bit keys); read and written only under g_tune_mu.
static std::mutex g_tune_mu;
static Tuning g_tuning[2];

Tuning tuning(int key_bytes) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_tuning[key_bytes == 8 ? 1 : 0];
}

static std::mutex g_ctx_mu;
static std::vector<DeviceCtx*> g_ctx;

// The status word of each device: a device global (zero when the code object
// is loaded), so that setting up a device allocates no memory.
static __device__ int g_status_word;

DeviceCtx* device_ctx(hipError_t* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_ctx_mu);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1, nullptr);
  if (g_ctx[dev]) return g_ctx[dev];
  DeviceCtx* c = new DeviceCtx();
  c->device = dev;
  e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
  // this device's copy of the status word (its address differs per device)
  if (e == hipSuccess) e = hipGetSymbolAddress(reinterpret_cast<void**>(&c->status), HIP_SYMBOL(g_status_word));
  if (e != hipSuccess) {
    delete c;
    *err = e;
    return nullptr;
  }
  g_ctx[dev] = c;
  return c;
}

static ss_status from_hip(hipError_t e) {
  if (e == hipSuccess) return SS_OK;
  if (e == hipErrorOutOfMemory) return SS_ENOMEM;
  return SS_EHIP;
}

template <class K>
static ss_status check_fixed(const void* keys, int32_t n, int64_t count, int64_t stride) {
  if (n < 0 || count < 0 || stride < 0) return SS_EINVAL;
  if (n > SS_MAX_N) return SS_ETOOBIG;
  if (stride < n) return SS_EINVAL;
  if (n <= 1 || count == 0) return 1;  // no-op
  if (keys == nullptr) return SS_EINVAL;
  if (reinterpret_cast<uintptr_t>(keys) % sizeof(K) != 0) return SS_EALIGN;
  if (count > (INT64_MAX / (stride > 0 ? stride : 1))) return SS_EINVAL;
  return SS_OK;
}

// W: the unsigned word of the key's width; map: the key type's order-preserving map.
template <class W>
static ss_status sort_small(void* keys_v, int32_t n, int64_t count, int64_t stride, KeyMap<W> map, hipStream_t s) {
  W* keys = static_cast<W*>(keys_v);
  ss_status st = check_fixed<W>(keys, n, count, stride);
  if (st == 1) return SS_OK;
  if (st != SS_OK) return st;
  hipError_t herr = hipSuccess;
  if (n <= SS_MAX_NETWORK_N) {
    if constexpr (sizeof(W) == 4)
      herr = launch_fixed_u32(keys, n, count, stride, map, s);
    else
      herr = launch_fixed_u64(keys, n, count, stride, map, s);
    return from_hip(herr);
  }
  if (n > SS_MAX_RSS_N) {
    if constexpr (sizeof(W) == 4)
      herr = launch_large_fixed_u32(keys, n, count, stride, map, s);
    else
      herr = launch_large_fixed_u64(keys, n, count, stride, map, s);
    return from_hip(herr);
  }
  DeviceCtx* c = device_ctx(&herr);
  if (!c) return from_hip(herr);
  if constexpr (sizeof(W) == 4)
    herr = launch_rss_fixed_u32(keys, n, count, stride, map, c->status, s);
  else
    herr = launch_rss_fixed_u64(keys, n, count, stride, map, c->status, s);
  return from_hip(herr);
}

static bool key_is_64(int32_t key_type) {
  return key_type == SS_KEY_U64 || key_type == SS_KEY_I64 || key_type == SS_KEY_F64;
}

template <class W>
static KeyMap<W> key_map(int32_t key_type) {
  switch (key_type) {
    case SS_KEY_I32:
    case SS_KEY_I64: return kSignedMap<W>;
    case SS_KEY_F32:
    case SS_KEY_F64: return kFloatMap<W>;
    default: return kUnsignedMap<W>;
  }
}

// vbytes: payload bytes per key (0 when vals is NULL, 4, or 8 with 64-bit keys).
static ss_status segmented(int32_t key_type, void* keys, void* vals, int32_t vbytes, const int32_t* offsets,
                           int32_t nseg, int32_t mode, hipStream_t s) {
  if (key_type < SS_KEY_U32 || key_type > SS_KEY_F64) return SS_EINVAL;
  if (mode < SS_MODE_AUTO || mode > SS_MODE_PLAIN) return SS_EINVAL;
  if (vbytes != 4 && vbytes != 8) return SS_EINVAL;
  if (vbytes == 8 && !key_is_64(key_type)) return SS_EINVAL;
  if (nseg < 0) return SS_EINVAL;
  if (nseg == 0) return SS_OK;
  if (keys == nullptr || offsets == nullptr) return SS_EINVAL;
  const size_t ksz = key_is_64(key_type) ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(keys) % ksz != 0) return SS_EALIGN;
  if (reinterpret_cast<uintptr_t>(offsets) % 4 != 0) return SS_EALIGN;
  if (vals && reinterpret_cast<uintptr_t>(vals) % vbytes != 0) return SS_EALIGN;
  const int vb = vals ? vbytes : 0;
  hipError_t herr = hipSuccess;
  DeviceCtx* c = device_ctx(&herr);
  if (!c) return from_hip(herr);
  if (key_is_64(key_type))
    return segmented_u64(c, static_cast<uint64_t*>(keys), vals, vb, offsets, nseg, key_map<uint64_t>(key_type), mode,
                         s);
  return segmented_u32(c, static_cast<uint32_t*>(keys), vals, vb, offsets, nseg, key_map<uint32_t>(key_type), mode, s);
}

// The no-allocation form of `segmented`: same checks, then the binning and
// persistent kernels launched directly on the device's fixed scratch array.
static_assert(kNoAllocMaxSeg == SS_NOALLOC_MAX_SEGMENTS, "header and library agree on the scratch limit");

static ss_status segmented_noalloc(int32_t key_type, void* keys, uint32_t* vals, const int32_t* offsets,
                                   int32_t nseg, hipStream_t s) {
  if (key_type < SS_KEY_U32 || key_type > SS_KEY_F64) return SS_EINVAL;
  if (nseg < 0) return SS_EINVAL;
  if (nseg > kNoAllocMaxSeg) return SS_ESCRATCH;
  if (nseg == 0) return SS_OK;
  if (keys == nullptr || offsets == nullptr) return SS_EINVAL;
  const size_t ksz = key_is_64(key_type) ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(keys) % ksz != 0) return SS_EALIGN;
  if (reinterpret_cast<uintptr_t>(offsets) % 4 != 0) return SS_EALIGN;
  if (vals && reinterpret_cast<uintptr_t>(vals) % 4 != 0) return SS_EALIGN;
  hipError_t herr = hipSuccess;
  DeviceCtx* c = device_ctx(&herr);
  if (!c) return from_hip(herr);
  SegBuffers b;
  herr = noalloc_buffers(c, &b);
  if (herr != hipSuccess) return from_hip(herr);
  const int vb = vals ? 4 : 0;
  if (key_is_64(key_type))
    return segmented_direct_u64(c, b, static_cast<uint64_t*>(keys), vals, vb, offsets, nseg,
                                key_map<uint64_t>(key_type), s);
  return segmented_direct_u32(c, b, static_cast<uint32_t*>(keys), vals, vb, offsets, nseg, key_map<uint32_t>(key_type),
                              s);
}

// --- tuning ----------------------------------------------------------------

struct TuneEntry {
  const char* name;
  int Tuning::*slot;
  int lo, hi;
  bool pow2_k;     // a bucket count: a power of two in [lo, hi]
  bool per_width;  // kept per key width ("u32.<name>" / "u64.<name>"); else one value
};

static const std::vector<TuneEntry>& tune_table() {
  static const std::vector<TuneEntry> table = {
      {"family", &Tuning::family, 0, 2, false, true},
      {"rss_k_small", nullptr, 4, 16, true, true},
      {"rss_k_mid", nullptr, 4, 32, true, true},
      {"rss_k_large", nullptr, 4, 64, true, true},
      {"rss_bound_tiny", &Tuning::rss_bound_tiny, 16, 32, false, true},
      {"rss_bound_small", &Tuning::rss_bound_small, 16, 64, false, true},
      {"rss_bound_mid", &Tuning::rss_bound_mid, 16, 128, false, true},
      {"rss_oversample", &Tuning::rss_oversample, 1, 4, false, true},
      {"fixed_apt", &Tuning::fixed_apt, 1, 4, false, true},
      {"fixed_half", &Tuning::fixed_half, 0, 0x1FFFC, false, true},
      {"fixed_wide", &Tuning::fixed_wide, 0, 0x1FFFC, false, true},
      {"fixed_wider", &Tuning::fixed_wider, 0, 0x1FFFC, false, true},
      {"rss_finish", &Tuning::rss_finish, 0, 1, false, true},
      {"persist_occ", &Tuning::persist_occ, 0, 16, false, false},
      {"rss_rounds", &Tuning::rss_rounds, 1, 64, false, false},
      {"interleave", &Tuning::interleave, 0, 1, false, false},
      {"persist_split", &Tuning::persist_split, 0, 1, false, false},
      {"net_mix", &Tuning::net_mix, 0, 1, false, false},
      {"rss_level_cap", &Tuning::rss_level_cap, 1, 8, false, false},
      {"large_sort", &Tuning::large_sort, 0, 1, false, false},
  };
  return table;
}

static int& slot_of(Tuning& t, const TuneEntry& e) {
  if (e.slot) return t.*(e.slot);
  // the three first-level bucket counts share an array
  return t.rss_k[e.name[6] == 's' ? 0 : (e.name[6] == 'm' ? 1 : 2)];
}

// name = "<knob>" (every key width) or "u32.<knob>" / "u64.<knob>" (one width
// of a per-width knob).  Returns the entry and the widths it addresses.
static const TuneEntry* find_knob(const char* name, bool& w32, bool& w64) {
  if (!name) return nullptr;
  w32 = w64 = true;
  if (std::strncmp(name, "u32.", 4) == 0) {
    w64 = false;
    name += 4;
  } else if (std::strncmp(name, "u64.", 4) == 0) {
    w32 = false;
    name += 4;
  }
  for (const TuneEntry& e : tune_table())
    if (std::strcmp(e.name, name) == 0) return (e.per_width || (w32 && w64)) ? &e : nullptr;
  return nullptr;
}

static bool valid_value(const TuneEntry& e, int64_t value, const Tuning& t) {
  if (value < e.lo || value > e.hi) return false;
  if (e.pow2_k && (value & (value - 1)) != 0) return false;
  if (e.slot == &Tuning::fixed_apt && value == 3) return false;
  if ((e.slot == &Tuning::fixed_half || e.slot == &Tuning::fixed_wide || e.slot == &Tuning::fixed_wider) &&
      (value & 3) != 0)
    return false;  // bits 2..16
  // a G-lane group holds at most 4G keys; bound_tiny <= bound_small <= bound_mid
  if (e.slot == &Tuning::rss_bound_mid && value < t.rss_bound_small) return false;
  if (e.slot == &Tuning::rss_bound_small && (value > t.rss_bound_mid || value < t.rss_bound_tiny)) return false;
  if (e.slot == &Tuning::rss_bound_tiny && value > t.rss_bound_small) return false;
  return true;
}

static ss_status set_tuning(const char* name, int64_t value) {
  bool w32, w64;
  const TuneEntry* e = find_knob(name, w32, w64);
  if (!e) return SS_ENOTUNE;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (int w = 0; w < 2; ++w)
    if ((w == 0 ? w32 : w64) && !valid_value(*e, value, g_tuning[w])) return SS_EINVAL;
  for (int w = 0; w < 2; ++w)
    if (w == 0 ? w32 : w64) slot_of(g_tuning[w], *e) = (int)value;
  return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" {

ss_status sort_small_u32(uint32_t* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint32_t>(keys, n, count, stride, kUnsignedMap<uint32_t>, static_cast<hipStream_t>(stream));
}
ss_status sort_small_i32(int32_t* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint32_t>(keys, n, count, stride, kSignedMap<uint32_t>, static_cast<hipStream_t>(stream));
}
ss_status sort_small_u64(uint64_t* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint64_t>(keys, n, count, stride, kUnsignedMap<uint64_t>, static_cast<hipStream_t>(stream));
}
ss_status sort_small_i64(int64_t* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint64_t>(keys, n, count, stride, kSignedMap<uint64_t>, static_cast<hipStream_t>(stream));
}
ss_status sort_small_f32(float* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint32_t>(keys, n, count, stride, kFloatMap<uint32_t>, static_cast<hipStream_t>(stream));
}
ss_status sort_small_f64(double* keys, int32_t n, int64_t count, int64_t stride, void* stream) {
  return sort_small<uint64_t>(keys, n, count, stride, kFloatMap<uint64_t>, static_cast<hipStream_t>(stream));
}

ss_status segmented_sort_u32(uint32_t* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg,
                             void* stream) {
  return segmented(SS_KEY_U32, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}
ss_status segmented_sort_i32(int32_t* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg,
                             void* stream) {
  return segmented(SS_KEY_I32, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}
ss_status segmented_sort_u64(uint64_t* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg,
                             void* stream) {
  return segmented(SS_KEY_U64, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}
ss_status segmented_sort_i64(int64_t* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg,
                             void* stream) {
  return segmented(SS_KEY_I64, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}

ss_status segmented_sort_f32(float* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg, void* stream) {
  return segmented(SS_KEY_F32, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}
ss_status segmented_sort_f64(double* keys, uint32_t* vals, const int32_t* offsets, int32_t nseg, void* stream) {
  return segmented(SS_KEY_F64, keys, vals, 4, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}

ss_status ss_segmented_sort(int32_t key_type, void* keys, uint32_t* vals, const int32_t* offsets,
                            int32_t nseg, int32_t mode, void* stream) {
  return segmented(key_type, keys, vals, 4, offsets, nseg, mode, static_cast<hipStream_t>(stream));
}

ss_status ss_segmented_sort_v(int32_t key_type, void* keys, void* vals, int32_t val_bytes, const int32_t* offsets,
                              int32_t nseg, int32_t mode, void* stream) {
  return segmented(key_type, keys, vals, val_bytes, offsets, nseg, mode, static_cast<hipStream_t>(stream));
}

ss_status segmented_sort_pairs_u64(uint64_t* keys, uint64_t* refs, const int32_t* offsets, int32_t nseg,
                                   void* stream) {
  return segmented(SS_KEY_U64, keys, refs, 8, offsets, nseg, SS_MODE_AUTO, static_cast<hipStream_t>(stream));
}

size_t ss_sort_workspace_bytes(int32_t key_type, int32_t val_bytes, int64_t n) {
  if (key_type < SS_KEY_U32 || key_type > SS_KEY_F64 || n < 0 || n > INT32_MAX) return 0;
  if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return 0;
  if (val_bytes == 8 && !key_is_64(key_type)) return 0;
  return devsort_workspace_bytes(n, key_is_64(key_type) ? 8 : 4, val_bytes);
}

ss_status ss_sort(int32_t key_type, void* keys, void* vals, int32_t val_bytes, int64_t n, void* workspace,
                  size_t workspace_bytes, void* stream) {
  if (key_type < SS_KEY_U32 || key_type > SS_KEY_F64) return SS_EINVAL;
  if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return SS_EINVAL;
  if (val_bytes == 8 && !key_is_64(key_type)) return SS_EINVAL;
  if ((vals == nullptr) != (val_bytes == 0)) return SS_EINVAL;
  if (n < 0 || n > INT32_MAX) return SS_EINVAL;
  if (n <= 1) return SS_OK;
  if (keys == nullptr || workspace == nullptr) return SS_EINVAL;
  const size_t ksz = key_is_64(key_type) ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(keys) % ksz != 0) return SS_EALIGN;
  if (vals && reinterpret_cast<uintptr_t>(vals) % (size_t)val_bytes != 0) return SS_EALIGN;
  if (workspace_bytes < devsort_workspace_bytes(n, (int)ksz, val_bytes)) return SS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = key_is_64(key_type)
                     ? devsort_u64(static_cast<uint64_t*>(keys), vals, val_bytes, n, workspace, workspace_bytes,
                                   key_map<uint64_t>(key_type), s)
                     : devsort_u32(static_cast<uint32_t*>(keys), vals, val_bytes, n, workspace, workspace_bytes,
                                   key_map<uint32_t>(key_type), s);
  return from_hip(e);
}

ss_status ss_segmented_sort_noalloc(int32_t key_type, void* keys, uint32_t* vals, const int32_t* offsets,
                                    int32_t nseg, void* stream) {
  return segmented_noalloc(key_type, keys, vals, offsets, nseg, static_cast<hipStream_t>(stream));
}

ss_status ss_device_status(void* stream, int32_t* out) {
  if (!out) return SS_EINVAL;
  hipError_t herr = hipSuccess;
  DeviceCtx* c = device_ctx(&herr);
  if (!c) return from_hip(herr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int value = 0;
  herr = hipStreamSynchronize(s);
  if (herr == hipSuccess) herr = hipMemcpy(&value, c->status, sizeof(int), hipMemcpyDeviceToHost);
  if (herr == hipSuccess) herr = hipMemset(c->status, 0, sizeof(int));
  if (herr == hipSuccess) herr = hipDeviceSynchronize();
  if (herr != hipSuccess) return SS_EHIP;
  *out = value;
  return SS_OK;
}

const char* ss_strerror(ss_status status) {
  switch (status) {
    case SS_OK: return "success";
    case SS_EINVAL: return "invalid argument (size, count, stride, pointer or offsets)";
    case SS_EALIGN: return "pointer not aligned to its element size";
    case SS_ETOOBIG: return "array or segment longer than 4096 keys";
    case SS_EHIP: return "HIP runtime error";
    case SS_ENOMEM: return "out of device memory";
    case SS_ENOTUNE: return "unknown tuning parameter or unreadable tuning file";
    case SS_ESCRATCH: return "batch exceeds the fixed working memory of the no-allocation entry point";
    case SS_EWORKSPACE: return "workspace smaller than ss_sort_workspace_bytes";
    default: return "unknown status";
  }
}

ss_status ss_stream_copy(void* dst, const void* src, int64_t bytes, void* stream) {
  if (bytes < 0) return SS_EINVAL;
  if (bytes == 0) return SS_OK;
  if (!dst || !src) return SS_EINVAL;
  if (reinterpret_cast<uintptr_t>(dst) % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 || bytes % 16 != 0)
    return SS_EALIGN;
  return from_hip(launch_stream_copy(dst, src, bytes, static_cast<hipStream_t>(stream)));
}

ss_status ss_set_tuning_value(const char* name, int64_t value) { return set_tuning(name, value); }

int64_t ss_get_tuning_value(const char* name) {
  bool w32, w64;
  const TuneEntry* e = find_knob(name, w32, w64);
  if (!e) return -1;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (w32 && w64) {  // one value for every width, or -2 if the widths differ
    const int a = slot_of(g_tuning[0], *e), b = slot_of(g_tuning[1], *e);
    return a == b ? a : -2;
  }
  return slot_of(g_tuning[w32 ? 0 : 1], *e);
}

// Minimal reader for a flat JSON object of integer values: {"a": 1, "b": 2}.
ss_status ss_load_tuning(const char* json_path) {
  if (!json_path) return SS_ENOTUNE;
  FILE* f = std::fopen(json_path, "rb");
  if (!f) return SS_ENOTUNE;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  size_t i = 0;
  auto skip = [&] {
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
  };
  skip();
  if (i >= text.size() || text[i] != '{') return SS_ENOTUNE;
  ++i;
  std::vector<std::pair<std::string, int64_t>> items;
  while (true) {
    skip();
    if (i < text.size() && text[i] == '}') break;
    if (i >= text.size() || text[i] != '"') return SS_ENOTUNE;
    size_t end = text.find('"', i + 1);
    if (end == std::string::npos) return SS_ENOTUNE;
    std::string key = text.substr(i + 1, end - i - 1);
    i = end + 1;
    skip();
    if (i >= text.size() || text[i] != ':') return SS_ENOTUNE;
    ++i;
    skip();
    // value: an integer, or any other JSON scalar/string which is skipped
    size_t vstart = i;
    if (i < text.size() && text[i] == '"') {
      size_t vend = text.find('"', i + 1);
      if (vend == std::string::npos) return SS_ENOTUNE;
      i = vend + 1;
    } else {
      while (i < text.size() && text[i] != ',' && text[i] != '}') ++i;
      std::string v = text.substr(vstart, i - vstart);
      while (!v.empty() && std::isspace((unsigned char)v.back())) v.pop_back();
      char* endp = nullptr;
      long long x = std::strtoll(v.c_str(), &endp, 10);
      if (!v.empty() && endp && *endp == '\0') items.emplace_back(key, (int64_t)x);
    }
    skip();
    if (i < text.size() && text[i] == ',') {
      ++i;
      continue;
    }
    skip();
    if (i < text.size() && text[i] == '}') break;
    return SS_ENOTUNE;
  }
  for (auto& kv : items) {
    ss_status st = set_tuning(kv.first.c_str(), kv.second);
    if (st == SS_EINVAL) return SS_EINVAL;
  }
  return SS_OK;
}

const char* ss_version(void) { return "smallsort 0.1 gfx950"; }

}  // extern "C"
