/*
 * smallsort.h -- C ABI of libsmallsort.so: sorting very many small independent
 * integer arrays on one AMD Instinct MI355X (gfx950).
 *
 * Method: "Engineering Faster Sorters for Small Sets of Items" (Bingmann,
 * Marianczuk, Sanders).  Arrays of 2..16 keys are sorted by branch-free
 * comparator networks held in registers (Section 2); arrays of 17..256 keys by
 * Register Sample Sort (Section 3), which splits them with sampled splitters
 * into buckets of at most 16 keys that are finished by networks; arrays of
 * 257..4096 keys by one work-group each, which sorts runs of 256 keys with
 * Register Sample Sort and merges them (the merge-sort use of the small
 * sorters that Section 5 proposes).
 *
 * Conventions shared by every call:
 *   - All pointers to keys, values and offsets are DEVICE pointers (memory from
 *     hipMalloc or any allocator returning device-accessible memory).  The
 *     caller owns every buffer; the library never frees or retains them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued asynchronously on it; no call synchronises the host,
 *     except ss_device_status and the SS_MODE_PLAIN baseline of
 *     ss_segmented_sort, which say so.
 *   - Sorting is in place and ascending (non-decreasing): the lower channel of
 *     every comparator receives the smaller key (Section 2.1).
 *   - Signed keys are ordered as two's-complement integers.  Float and double
 *     keys are ordered by IEEE 754 totalOrder: -NaN < -inf < ... < -0 < +0 <
 *     ... < +inf < +NaN (NaNs of one sign by their payload bits).  Without NaNs
 *     this is non-decreasing order under the float comparison, with -0 placed
 *     before +0 (the paper compares floats with the CPU's compare instruction,
 *     Section 2.2; a total order keeps every result unique).
 *   - With a payload (`vals` != NULL, a uint32 array parallel to the keys) the
 *     (key, value) pairs are permuted together.  Equal keys may come out in
 *     any order relative to each other (networks are not stable), so the
 *     payload of equal keys is only defined as a multiset.
 *   - Return values are ss_status codes; SS_OK is 0, errors are negative.
 *     Argument errors are detected on the host before anything is enqueued.
 *     Errors that depend on device data (a segment longer than 4096 keys, a
 *     decreasing offset) are recorded in a per-device status word, read with
 *     ss_device_status; the affected segment is left unsorted.
 *   - Working memory of the segmented path (counters, size-class lists,
 *     cached graph) is allocated per (device, stream) on first use.  When a
 *     larger batch arrives its segment list is grown in stream order
 *     (hipFreeAsync / hipMallocAsync on the call's stream, which is the only
 *     stream that uses it), with no host or device synchronisation; calls of
 *     the same or smaller shape allocate nothing.  It is kept until the
 *     process ends (about 5 bytes per segment of the largest batch plus 80 KB
 *     per stream), so a caller should not churn through short-lived streams.
 *   - Calls are thread-safe.  Segmented sorts on different streams use
 *     separate working memory and may overlap on the device; calls on one
 *     stream are ordered by that stream.
 */
#ifndef SMALLSORT_H
#define SMALLSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ss_status;

#define SS_OK        0
#define SS_EINVAL   (-1)  /* bad size, count, stride or pointer */
#define SS_EALIGN   (-2)  /* a pointer not aligned to its element size */
#define SS_ETOOBIG  (-3)  /* an array or segment longer than SS_MAX_N */
#define SS_EHIP     (-4)  /* a HIP runtime call failed */
#define SS_ENOMEM   (-5)  /* working memory could not be allocated */
#define SS_ENOTUNE  (-6)  /* unknown tuning name or unreadable tuning file */
#define SS_ESCRATCH (-7)  /* batch larger than the no-allocation entry point's scratch */
#define SS_EWORKSPACE (-8)  /* workspace smaller than ss_sort_workspace_bytes */

#define SS_MAX_NETWORK_N 16   /* largest array sorted by a network alone */
#define SS_MAX_RSS_N    256   /* largest array sorted by Register Sample Sort alone */
#define SS_MAX_N       4096   /* largest array or segment */

/* Key type codes for the generic entry points. */
#define SS_KEY_U32 0
#define SS_KEY_I32 1
#define SS_KEY_U64 2
#define SS_KEY_I64 3
#define SS_KEY_F32 4
#define SS_KEY_F64 5

/* Execution modes for ss_segmented_sort. */
#define SS_MODE_AUTO       0  /* persistent kernel, replayed from a cached hipGraph */
#define SS_MODE_PERSISTENT 1  /* persistent kernel, launched directly (no graph) */
#define SS_MODE_PLAIN      2  /* one ordinary launch per size class */

/*
 * Fixed layout (Sections 2 and 3; the ArrayInRow arrangement of Section 4.1):
 * array i occupies keys[i*stride, i*stride + n) for 0 <= i < count.  Entries
 * [n, stride) of each row are neither read nor written.
 *   n:      0..4096.  n <= 1 or count == 0 is a no-op returning SS_OK.
 *           2..16 use one comparator network per array; 17..256 use
 *           Register Sample Sort; 257..4096 one work-group per array (runs of
 *           256 keys by Register Sample Sort, merged in LDS).
 *   stride: >= n (in keys).  count * stride keys must be addressable.
 * Errors: SS_EINVAL for n < 0, count < 0, stride < n or keys == NULL with
 * count > 0; SS_ETOOBIG for n > 4096; SS_EALIGN if keys is not aligned to the
 * key size; SS_EHIP if a launch fails.
 */
ss_status sort_small_u32(uint32_t *keys, int32_t n, int64_t count, int64_t stride, void *stream);
ss_status sort_small_i32(int32_t *keys, int32_t n, int64_t count, int64_t stride, void *stream);
ss_status sort_small_u64(uint64_t *keys, int32_t n, int64_t count, int64_t stride, void *stream);
ss_status sort_small_i64(int64_t *keys, int32_t n, int64_t count, int64_t stride, void *stream);
ss_status sort_small_f32(float *keys, int32_t n, int64_t count, int64_t stride, void *stream);
ss_status sort_small_f64(double *keys, int32_t n, int64_t count, int64_t stride, void *stream);

/*
 * Segmented layout (CSR): segment i is [offsets[i], offsets[i+1]) for
 * 0 <= i < nseg; `offsets` is a device int32 array of nseg+1 non-decreasing
 * entries (offsets[0] need not be 0).  Segment sizes 0..4096; sizes 0 and 1
 * are no-ops.  The batch is binned by segment size (Section 5's proposal of
 * solving base cases in batches of equal size) and sorted by one persistent
 * launch: networks for 2..16 keys, Register Sample Sort for 17..256, one
 * work-group per segment of 257..4096 keys.
 *   vals: NULL (keys only) or a device uint32 array indexed like keys.
 * Errors: SS_EINVAL for nseg < 0 or a NULL pointer with nseg > 0; SS_EALIGN
 * for misaligned pointers; SS_ENOMEM / SS_EHIP from working memory or
 * launches.  Segments longer than 4096 keys or with decreasing offsets are
 * skipped and flagged in the device status word (SS_ETOOBIG / SS_EINVAL).
 */
ss_status segmented_sort_u32(uint32_t *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);
ss_status segmented_sort_i32(int32_t *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);
ss_status segmented_sort_u64(uint64_t *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);
ss_status segmented_sort_i64(int64_t *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);
ss_status segmented_sort_f32(float *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);
ss_status segmented_sort_f64(double *keys, uint32_t *vals, const int32_t *offsets, int32_t nseg, void *stream);

/*
 * Generic segmented entry point: key_type is an SS_KEY_* code, mode an
 * SS_MODE_* code.  Same layout, ownership and errors as segmented_sort_*;
 * SS_EINVAL for an unknown key_type or mode.  SS_MODE_PLAIN is the
 * per-size-class baseline the persistent form is measured against: it reads
 * the class counts back to the host to size one launch per class, so it
 * synchronises `stream` in the middle of the call (the other modes do not).
 */
ss_status ss_segmented_sort(int32_t key_type, void *keys, uint32_t *vals, const int32_t *offsets,
                            int32_t nseg, int32_t mode, void *stream);

/*
 * Segmented sort with a payload of either width: vals is NULL (keys only) or a
 * device array parallel to keys of val_bytes = 4 (uint32) or 8 (uint64; 64-bit
 * key types only) per key.  With 64-bit keys and 8-byte values this sorts the
 * paper's items, a 64-bit key with a 64-bit reference (Section 2.2), stored as
 * two parallel arrays.  Errors as ss_segmented_sort; SS_EINVAL for another
 * val_bytes or for 8-byte values with 32-bit keys; SS_EALIGN if vals is not
 * aligned to val_bytes.
 */
ss_status ss_segmented_sort_v(int32_t key_type, void *keys, void *vals, int32_t val_bytes, const int32_t *offsets,
                              int32_t nseg, int32_t mode, void *stream);
/* ss_segmented_sort_v(SS_KEY_U64, keys, refs, 8, offsets, nseg, SS_MODE_AUTO, stream). */
ss_status segmented_sort_pairs_u64(uint64_t *keys, uint64_t *refs, const int32_t *offsets, int32_t nseg,
                                   void *stream);

/*
 * One large array sorted on the device, with the small sorters as its base
 * case (the paper's use of them inside Quicksort and IPS4o, Sections 4.4 and
 * 4.6, and the batching of base cases by size proposed in Section 5): sample
 * sort partitions with about 1536 (32-bit keys) or 1024 (64-bit keys) keys per
 * bucket and equality buckets for repeated splitters, then one segmented sort
 * of every bucket; a bucket still above 4096 keys is partitioned again.
 *   keys:  n keys of key_type (SS_KEY_*), sorted in place (ascending; same
 *          order as the other calls).  n: 0 .. 2^31 - 1.
 *   vals:  NULL with val_bytes = 0, or a payload of val_bytes = 4 or 8 (8: 64-bit
 *          keys only) per key, permuted with the keys; the order of equal keys
 *          is unspecified.
 *   workspace: device memory of at least ss_sort_workspace_bytes(key_type,
 *          val_bytes, n) bytes (about n * (key + payload bytes) plus 3%),
 *          owned by the caller; the call allocates nothing.
 * Unlike the other calls it synchronises `stream` (between partition levels
 * the host reads how many buckets need another level).
 * Errors: SS_EINVAL for a bad key_type, val_bytes, n or pointer; SS_EALIGN for
 * misaligned keys or vals; SS_EWORKSPACE if the workspace is too small;
 * SS_EHIP if a launch fails.
 */
size_t ss_sort_workspace_bytes(int32_t key_type, int32_t val_bytes, int64_t n);
ss_status ss_sort(int32_t key_type, void *keys, void *vals, int32_t val_bytes, int64_t n, void *workspace,
                  size_t workspace_bytes, void *stream);

/*
 * No-allocation form of ss_segmented_sort, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same layout, ownership, results and device status
 * reporting as ss_segmented_sort with SS_MODE_PERSISTENT; it calls no
 * hipMalloc, hipFree or other allocating routine.  Its working memory is one
 * fixed array per device in the library's code object (64 MiB + 88 KiB, held
 * until the process ends), looked up on the first call on each device.
 *   nseg: 0..SS_NOALLOC_MAX_SEGMENTS; a larger batch returns SS_ESCRATCH
 *         before anything is enqueued.
 * Every call on one device shares that array: calls that overlap on the
 * device (calls on different streams, or from different host threads, not
 * ordered by the caller) race and give undefined results.  Calls ordered on
 * one stream are safe; nothing carries over from one call to the next.
 * Errors: as ss_segmented_sort, plus SS_ESCRATCH.
 */
#define SS_NOALLOC_MAX_SEGMENTS (1 << 24)
ss_status ss_segmented_sort_noalloc(int32_t key_type, void *keys, uint32_t *vals, const int32_t *offsets,
                                    int32_t nseg, void *stream);

/*
 * Reads the current device's status word after synchronising `stream`, stores
 * it in *out (SS_OK, or the first error code recorded by a kernel) and clears
 * it.  Returns SS_EINVAL if out is NULL, SS_EHIP if the copy fails.
 */
ss_status ss_device_status(void *stream, int32_t *out);

/* A static, human-readable description of a status code (never NULL). */
const char *ss_strerror(ss_status status);

/*
 * Tuning parameters (variant choices found by the autotuner).  The first
 * thirteen are kept per key width: "<name>" sets both widths, "u32.<name>" or
 * "u64.<name>" one of them (32-bit keys: uint32, int32, float; 64-bit keys:
 * uint64, int64, double); getting "<name>" returns -2 when the widths differ.
 *   "family"       n <= 16: 0 = fewest-comparator networks, 1 = Bose-Nelson
 *                  networks, 2 = insertion sort (the paper's baseline)
 *   "rss_k_small"  buckets (4, 8 or 16; splitters + 1) of the first Register
 *                  Sample Sort level for arrays of the 16-lane class
 *   "rss_k_mid"    same for the 32-lane class (4, 8, 16 or 32)
 *   "rss_k_large"  same for the 64-lane class (4, 8, 16, 32 or 64)
 *   "rss_bound_tiny" arrays of 17..bound_tiny keys are sorted by 8 lanes
 *                  (16..32; 16 = none)
 *   "rss_bound_small" arrays of bound_tiny+1..bound_small keys by 16 lanes
 *                  (16..64, default 64; at most 4 keys per lane)
 *   "rss_bound_mid" arrays of bound_small+1..bound_mid keys by 32 lanes
 *                  (bound_small..128, default 128), larger ones by 64 lanes
 *   "rss_oversample" oversampling factor a of the Register Sample Sort levels
 *                  with 4 buckets (1..4, default 3: the paper's "332")
 *   "fixed_apt"    arrays per thread of the fixed-layout network kernels (1, 2
 *                  or 4; reduced where the tile would not fit 32 KiB of LDS)
 *   "fixed_half"   bit mask over n = 2..16 (bit n, 0..0x1FFFC, default 0):
 *                  where one array per thread is used, arrays of n keys are
 *                  staged by 128-thread work-groups (half the LDS tile of the
 *                  256-thread form)
 *   "fixed_wide"   same form of mask: arrays of n keys are staged by
 *                  512-thread work-groups over tiles of 256 arrays (each
 *                  thread moves half as many chunks); takes precedence over
 *                  "fixed_half"
 *   "fixed_wider"  same, with 1024-thread work-groups (a quarter of the
 *                  chunks per thread); takes precedence over both.  The two
 *                  wide forms apply to the network families only (with
 *                  family 2, insertion sort, their bits are ignored)
 *   "rss_finish"   how Register Sample Sort finishes its buckets of 2..16
 *                  keys: 0 = one network per bucket (Section 3, default),
 *                  1 = rank counting (each key counts the smaller keys of its
 *                  bucket and moves once; cheaper where an exchange moves
 *                  64-bit keys or payloads)
 *   "persist_occ"  work-groups per CU of the persistent grid (0 = as many as
 *                  fit, 1..16)
 *   "rss_rounds"   most rounds of lane groups per RSS tile in segmented sorts
 *                  (1..64; fewer when a size class has few segments)
 *   "interleave"   1: the persistent kernel alternates RSS and network tiles
 *   "persist_split" 1: a persistent kernel for the network classes, then one
 *                  per RSS size class (each with only its own code and
 *                  registers); 0: a single persistent kernel for every class
 *   "net_mix"      1: in the persistent forms, segments of 2..16 keys are
 *                  sorted in batch order, 64 per tile of mixed sizes: the
 *                  tile's keys are read and written as one run of consecutive
 *                  elements through LDS (neighbouring segments share cache
 *                  lines), each lane running the network of the tile's
 *                  largest segment; 0: one class per size, each with its
 *                  exact network, one segment per lane read in place.  The
 *                  plain form always uses one class per size.
 *   "rss_level_cap" levels of Register Sample Sort (1..8, default 8) after
 *                  which a bucket still above 16 keys is finished by a
 *                  rank-counting sort (each key placed at the number of keys
 *                  that precede it); lower values exist to test and measure
 *                  that fallback.
 *   "large_sort"   1: arrays of more than 16 keys are sorted by insertion sort
 *                  (the paper's IS+SN hybrid, Section 4.6); 0: Register Sample
 *                  Sort (default)
 * ss_set_tuning_value returns SS_ENOTUNE for an unknown name (or a width
 * prefix on a knob that has one value), SS_EINVAL for a value out of range.
 * ss_get_tuning_value returns -1 for an unknown name.
 * ss_load_tuning reads a flat JSON object {"name": integer, ...} with these
 * names (other keys are ignored); SS_ENOTUNE if the file cannot be read or
 * parsed.  Settings are process-wide and apply to later calls.
 */
ss_status ss_set_tuning_value(const char *name, int64_t value);
int64_t ss_get_tuning_value(const char *name);
ss_status ss_load_tuning(const char *json_path);

/*
 * Streaming device-to-device copy of `bytes` bytes from src to dst, with the
 * access pattern of the fixed-layout sorting kernels (16-byte nontemporal
 * loads and stores, consecutive lanes on consecutive chunks).  It is the
 * practical ceiling a read-once / write-once kernel reaches on this device,
 * against which the sorts are measured.  dst and src are device pointers of
 * non-overlapping buffers.  Errors: SS_EINVAL for bytes < 0 or a NULL pointer
 * with bytes > 0; SS_EALIGN unless both pointers and bytes are multiples of 16.
 */
ss_status ss_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* Library version string, e.g. "smallsort 0.1 gfx950". */
const char *ss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMALLSORT_H */
