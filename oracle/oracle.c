/*
 * CPU oracle for batched small-array sorting.  TEST INFRASTRUCTURE ONLY:
 * it is called by tests/, by the smoke check and by the bench's CPU-baseline
 * leg, never by the library itself.  It shares no code with the GPU path.
 *
 * What it computes.  Section 2.1 of "Engineering Faster Sorters for Small
 * Sets of Items" (Bingmann, Marianczuk, Sanders) defines the result of a
 * sorting network: the channels end holding a permutation of the input in
 * non-decreasing order.  Register Sample Sort (Section 3) reaches the same
 * result.  So the oracle is simply "sort each array ascending":
 *
 *   - insertion sort for n <= 16 (the textbook form the paper benchmarks the
 *     networks against, Section 4.2, variant "IS Def");
 *   - a separate top-down merge sort with a scratch buffer for n > 16.
 *
 * Both are stable, so with a payload the oracle keeps equal keys in input
 * order.  (Networks are not stable; callers compare payloads exactly only
 * when the keys of a segment are distinct.)
 *
 * Key types: uint32, int32, uint64, int64, compared natively (signed keys in
 * two's-complement order), and float / double, ordered by IEEE 754
 * totalOrder (the paper compares floats with the CPU's compare, Section 2.2;
 * a total order keeps every result unique): a key with the sign bit set
 * precedes one without; among keys with the sign bit clear the smaller
 * magnitude (exponent and significand bits) comes first, among keys with it
 * set the larger magnitude.  So -NaN < -inf < ... < -0 < +0 < ... < +inf <
 * +NaN.  The payload, when present, is an array parallel to the keys of
 * uint32 (names without a suffix) or uint64 (names ending in _v64); NULL
 * means keys only.
 *
 * Layouts:
 *   fixed:     array i occupies keys[i*stride .. i*stride+n); entries
 *              [n, stride) of each row are left untouched.
 *   segmented: segment i occupies [offsets[i], offsets[i+1]) (CSR, int32).
 *
 * Error behaviour: none of these functions validates its arguments; the
 * callers (Python wrappers in this folder) check shapes first.  merge sort
 * returns -1 if its scratch allocation fails, 0 otherwise.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* "a precedes b" for each key type. */
static inline int lt_u32(uint32_t a, uint32_t b) { return a < b; }
static inline int lt_i32(int32_t a, int32_t b) { return a < b; }
static inline int lt_u64(uint64_t a, uint64_t b) { return a < b; }
static inline int lt_i64(int64_t a, int64_t b) { return a < b; }

/* totalOrder on sign and magnitude, as described above. */
static inline int lt_f32(float a, float b) {
    uint32_t x, y;
    memcpy(&x, &a, sizeof x);
    memcpy(&y, &b, sizeof y);
    const uint32_t sx = x >> 31, sy = y >> 31;
    const uint32_t mx = x & 0x7FFFFFFFu, my = y & 0x7FFFFFFFu;
    if (sx != sy) return sx > sy;      /* sign set first */
    return sx ? mx > my : mx < my;     /* negatives: larger magnitude first */
}
static inline int lt_f64(double a, double b) {
    uint64_t x, y;
    memcpy(&x, &a, sizeof x);
    memcpy(&y, &b, sizeof y);
    const uint64_t sx = x >> 63, sy = y >> 63;
    const uint64_t mx = x & 0x7FFFFFFFFFFFFFFFull, my = y & 0x7FFFFFFFFFFFFFFFull;
    if (sx != sy) return sx > sy;
    return sx ? mx > my : mx < my;
}

/* One definition per (key type, payload type), stamped by this macro.  T is
 * the key type, S the suffix of the exported names, VT the payload type, LT
 * the key order. */
#define ORACLE_DEFINE(T, S, VT, LT)                                           \
                                                                              \
/* Insertion sort: grow a sorted prefix; move each new item left past every  \
 * key it strictly precedes (so equal keys keep input order). */             \
void oracle_insertion_sort_##S(T *keys, VT *vals, int64_t n)                  \
{                                                                             \
    for (int64_t i = 1; i < n; ++i) {                                         \
        T k = keys[i];                                                        \
        VT v = vals ? vals[i] : 0;                                            \
        int64_t j = i;                                                        \
        while (j > 0 && LT(k, keys[j - 1])) {                                 \
            keys[j] = keys[j - 1];                                            \
            if (vals) vals[j] = vals[j - 1];                                  \
            --j;                                                              \
        }                                                                     \
        keys[j] = k;                                                          \
        if (vals) vals[j] = v;                                                \
    }                                                                         \
}                                                                             \
                                                                              \
/* Top-down merge sort of keys[lo, hi) using tk/tv as scratch of the same    \
 * extent.  Ties take the left run first, which keeps the sort stable. */    \
static void merge_rec_##S(T *keys, VT *vals, T *tk, VT *tv,                   \
                          int64_t lo, int64_t hi)                             \
{                                                                             \
    if (hi - lo < 2) return;                                                  \
    int64_t mid = lo + (hi - lo) / 2;                                         \
    merge_rec_##S(keys, vals, tk, tv, lo, mid);                               \
    merge_rec_##S(keys, vals, tk, tv, mid, hi);                               \
    int64_t a = lo, b = mid, o = lo;                                          \
    while (a < mid && b < hi) {                                               \
        if (LT(keys[b], keys[a])) {                                           \
            tk[o] = keys[b]; if (vals) tv[o] = vals[b]; ++b;                  \
        } else {                                                              \
            tk[o] = keys[a]; if (vals) tv[o] = vals[a]; ++a;                  \
        }                                                                     \
        ++o;                                                                  \
    }                                                                         \
    while (a < mid) { tk[o] = keys[a]; if (vals) tv[o] = vals[a]; ++a; ++o; } \
    while (b < hi)  { tk[o] = keys[b]; if (vals) tv[o] = vals[b]; ++b; ++o; } \
    for (int64_t i = lo; i < hi; ++i) {                                       \
        keys[i] = tk[i];                                                      \
        if (vals) vals[i] = tv[i];                                            \
    }                                                                         \
}                                                                             \
                                                                              \
int oracle_merge_sort_##S(T *keys, VT *vals, int64_t n)                       \
{                                                                             \
    if (n < 2) return 0;                                                      \
    T *tk = (T *)malloc((size_t)n * sizeof(T));                               \
    VT *tv = vals ? (VT *)malloc((size_t)n * sizeof(VT)) : NULL;              \
    if (!tk || (vals && !tv)) { free(tk); free(tv); return -1; }              \
    merge_rec_##S(keys, vals, tk, tv, 0, n);                                  \
    free(tk);                                                                 \
    free(tv);                                                                 \
    return 0;                                                                 \
}                                                                             \
                                                                              \
/* Sort one array: insertion sort up to 16 items, merge sort above. */       \
int oracle_sort_##S(T *keys, VT *vals, int64_t n)                             \
{                                                                             \
    if (n <= 16) { oracle_insertion_sort_##S(keys, vals, n); return 0; }      \
    return oracle_merge_sort_##S(keys, vals, n);                              \
}                                                                             \
                                                                              \
int oracle_sort_fixed_##S(T *keys, int64_t n, int64_t count, int64_t stride)  \
{                                                                             \
    for (int64_t i = 0; i < count; ++i)                                       \
        if (oracle_sort_##S(keys + i * stride, NULL, n)) return -1;           \
    return 0;                                                                 \
}                                                                             \
                                                                              \
int oracle_sort_segments_##S(T *keys, VT *vals, const int32_t *offsets,       \
                             int64_t nseg)                                    \
{                                                                             \
    for (int64_t i = 0; i < nseg; ++i) {                                      \
        int64_t lo = offsets[i], hi = offsets[i + 1];                         \
        if (oracle_sort_##S(keys + lo, vals ? vals + lo : NULL, hi - lo))     \
            return -1;                                                        \
    }                                                                         \
    return 0;                                                                 \
}

ORACLE_DEFINE(uint32_t, u32, uint32_t, lt_u32)
ORACLE_DEFINE(int32_t, i32, uint32_t, lt_i32)
ORACLE_DEFINE(uint64_t, u64, uint32_t, lt_u64)
ORACLE_DEFINE(int64_t, i64, uint32_t, lt_i64)
ORACLE_DEFINE(float, f32, uint32_t, lt_f32)
ORACLE_DEFINE(double, f64, uint32_t, lt_f64)
/* 64-bit keys with a 64-bit payload (the paper's key + reference items). */
ORACLE_DEFINE(uint64_t, u64_v64, uint64_t, lt_u64)
ORACLE_DEFINE(int64_t, i64_v64, uint64_t, lt_i64)
ORACLE_DEFINE(double, f64_v64, uint64_t, lt_f64)
