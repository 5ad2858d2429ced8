"""Pins for the CPU oracle (no GPU).

The oracle defines the result every GPU path must reproduce bit-exactly:
each array sorted non-decreasing (paper, Section 2.1).  These tests tie it to
things other than itself:

  * brute force -- every permutation of 0..n-1 (n <= 8) must come out as the
    identity; every word over {0,1,2,3}^n (n <= 8) must come out with the same
    value counts in order (a counting-sort construction);
  * Python's ``sorted`` on exact integers for all words over the extreme values
    of each key type;
  * numpy's sort / stable argsort on random inputs for every n up to 256;
  * the paper's own permutation check (Section 4.1): the product of (z - a_i)
    modulo a large prime is unchanged by sorting;
  * layout invariants (stride gaps untouched, CSR segments independent).

``test_planted_mistakes`` compiles copies of oracle.c with one plausible
mistake each and asserts that some pin fails for every one of them.
"""
import itertools
import shutil

import numpy as np
import pytest

import oracle
from oracle import build as oracle_build

TYPES = [np.uint32, np.int32, np.uint64, np.int64]
RNG_SEED = 12345


def _rand(dtype, size, rng):
    info = np.iinfo(dtype)
    return rng.integers(info.min, info.max, size=size, dtype=dtype, endpoint=True)


def _counting_sorted(words, nvals):
    """Rows rebuilt from value counts: c_0 zeros, then c_1 ones, ..."""
    out = np.empty_like(words)
    for r in range(words.shape[0]):
        counts = np.bincount(words[r], minlength=nvals)
        out[r] = np.repeat(np.arange(nvals, dtype=words.dtype), counts)
    return out


# ---------------------------------------------------------------- the pins --

def pin_permutations(lib, max_n=8):
    for n in range(1, max_n + 1):
        perms = np.array(list(itertools.permutations(range(n))), dtype=np.int32).reshape(-1, n)
        ident = np.arange(n, dtype=np.int32)
        got = oracle.sort_fixed(perms.reshape(-1), n, perms.shape[0], n, lib=lib).reshape(-1, n)
        assert (got == ident).all(), f"permutations n={n} (dispatching sort)"
        step = 1 if n <= 7 else 7  # merge sort per row: thin the n=8 set
        for p in perms[::step]:
            k, _ = oracle.merge_sort(p, lib=lib)
            assert (k == ident).all(), f"merge sort of permutation {p}"
            k, _ = oracle.insertion_sort(p, lib=lib)
            assert (k == ident).all(), f"insertion sort of permutation {p}"


def pin_small_words(lib, max_n=8):
    for n in range(1, max_n + 1):
        words = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.uint32)
        want = _counting_sorted(words, 4)
        got = oracle.sort_fixed(words.reshape(-1), n, words.shape[0], n, lib=lib).reshape(-1, n)
        assert (got == want).all(), f"words over 0..3, n={n}"
        if n in (5, 8):
            for w, ww in zip(words[::97], want[::97]):
                assert (oracle.merge_sort(w, lib=lib)[0] == ww).all(), f"merge sort word {w}"


def pin_extremes(lib):
    for dt in TYPES:
        info = np.iinfo(dt)
        vals = sorted({int(info.min), int(info.min) + 1, 0, 1, int(info.max) - 1, int(info.max)}
                      | ({-1} if info.min < 0 else set()))
        for n in range(1, 5):
            for w in itertools.product(vals, repeat=n):
                want = sorted(w)
                a = np.array(w, dtype=dt)
                for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                    got = [int(x) for x in f(a, lib=lib)[0]]
                    assert got == want, f"{dt.__name__} {w} via {f.__name__}"


def pin_random_vs_numpy(lib):
    rng = np.random.default_rng(RNG_SEED)
    for dt in TYPES:
        for n in list(range(0, 40)) + [63, 64, 65, 100, 127, 128, 129, 200, 255, 256]:
            for _ in range(3):
                a = _rand(dt, n, rng)
                want = np.sort(a, kind="stable")
                for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                    assert (f(a, lib=lib)[0] == want).all(), f"{dt.__name__} n={n} {f.__name__}"


def pin_payload_stable(lib):
    """With a payload the pairs follow the keys; equal keys keep input order."""
    rng = np.random.default_rng(RNG_SEED + 1)
    for dt in TYPES:
        for n in (2, 5, 16, 17, 40, 256):
            for few in (False, True):
                a = (rng.integers(0, 4, size=n).astype(dt) if few else _rand(dt, n, rng))
                v = np.arange(n, dtype=np.uint32)
                order = np.argsort(a, kind="stable")
                for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                    k, vv = f(a, v, lib=lib)
                    assert (k == a[order]).all() and (vv == v[order]).all(), \
                        f"{dt.__name__} n={n} few={few} {f.__name__}"


def _perm_fingerprint(values, z, p):
    prod = 1
    for a in values:
        prod = (prod * ((z - int(a)) % p)) % p
    return prod


def pin_permutation_product(lib):
    """Section 4.1's check: prod (z - a_i) mod p is invariant under sorting."""
    p = (1 << 61) - 1  # a Mersenne prime
    rng = np.random.default_rng(RNG_SEED + 2)
    for dt in TYPES:
        for n in (3, 16, 31, 256):
            a = _rand(dt, n, rng)
            z = 0x1234567
            v = _perm_fingerprint(a, z, p)
            while v == 0:
                z += 1
                v = _perm_fingerprint(a, z, p)
            for f in (oracle.insertion_sort, oracle.merge_sort):
                k = f(a, lib=lib)[0]
                assert _perm_fingerprint(k, z, p) == v, f"permutation check {dt.__name__} n={n}"
                assert (k[1:] >= k[:-1]).all(), f"sortedness {dt.__name__} n={n}"


def pin_fixed_stride(lib):
    rng = np.random.default_rng(RNG_SEED + 3)
    for dt in TYPES:
        for n, stride in ((4, 4), (5, 7), (16, 19), (20, 32)):
            count = 33
            a = _rand(dt, count * stride, rng)
            got = oracle.sort_fixed(a, n, count, stride, lib=lib).reshape(count, stride)
            src = a.reshape(count, stride)
            assert (got[:, n:] == src[:, n:]).all(), "stride gap touched"
            assert (got[:, :n] == np.sort(src[:, :n], axis=1)).all(), f"fixed n={n} stride={stride}"


def pin_segments(lib):
    rng = np.random.default_rng(RNG_SEED + 4)
    for dt in TYPES:
        sizes = np.array([0, 1, 2, 0, 17, 256, 3, 0, 16, 100, 1], dtype=np.int64)
        base = 5  # offsets need not start at zero
        off = (np.concatenate([[0], np.cumsum(sizes)]) + base).astype(np.int32)
        a = _rand(dt, int(off[-1]) + 4, rng)
        v = np.arange(a.size, dtype=np.uint32)
        k, vv = oracle.sort_segments(a, off, v, lib=lib)
        assert (k[:base] == a[:base]).all() and (k[off[-1]:] == a[off[-1]:]).all()
        for i in range(sizes.size):
            lo, hi = off[i], off[i + 1]
            order = np.argsort(a[lo:hi], kind="stable")
            assert (k[lo:hi] == a[lo:hi][order]).all(), f"segment {i}"
            assert (vv[lo:hi] == v[lo:hi][order]).all(), f"segment payload {i}"


# --- float keys (IEEE 754 totalOrder) and 64-bit payloads ------------------

FLOATS = [np.float32, np.float64]


def _finite_floats(dt, size, rng):
    """Finite values over many magnitudes, both signs, no -0.0 and no NaN."""
    x = rng.standard_normal(size) * np.exp2(rng.integers(-60, 60, size=size))
    x = x.astype(dt)
    x[x == 0] = dt(1.0)
    return x


def pin_float_vs_numpy(lib):
    """Without signed zeros and NaNs, totalOrder is the order of the float
    compare: numpy's sort."""
    rng = np.random.default_rng(RNG_SEED + 5)
    for dt in FLOATS:
        for n in list(range(0, 20)) + [31, 64, 65, 129, 256]:
            a = _finite_floats(dt, n, rng)
            if n > 3:
                a[rng.integers(0, n, size=2)] = [np.inf, -np.inf]
            want = np.sort(a, kind="stable")
            for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                assert (f(a, lib=lib)[0] == want).all(), f"{dt.__name__} n={n} {f.__name__}"
        count, n = 50, 12
        a = _finite_floats(dt, count * n, rng)
        got = oracle.sort_fixed(a, n, count, n, lib=lib).reshape(count, n)
        assert (got == np.sort(a.reshape(count, n), axis=1)).all()


def pin_float_signed_zeros_and_infinities(lib):
    """Every word of length <= 4 over special values against Python's sorted,
    with -0.0 placed before +0.0 (the float value, then the sign of the zero)."""
    import math
    specials = [-np.inf, -2.5, -0.0, 0.0, 1.0, np.inf]
    key = lambda x: (x, math.copysign(1.0, x))  # noqa: E731
    for dt in FLOATS:
        for n in range(1, 5):
            for w in itertools.product(specials, repeat=n):
                want = sorted(w, key=key)
                a = np.array(w, dtype=dt)
                for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                    got = f(a, lib=lib)[0]
                    assert [(float(x), math.copysign(1.0, x)) for x in got] == [key(x) for x in want], \
                        f"{dt.__name__} {w} via {f.__name__}"


def pin_float_nans_at_the_ends(lib):
    """NaNs with the sign bit set come first, the others last; the finite
    middle is in float order."""
    rng = np.random.default_rng(RNG_SEED + 6)
    for dt in FLOATS:
        for n in (5, 16, 40, 200):
            a = _finite_floats(dt, n, rng)
            pos = rng.choice(n, size=4, replace=False)
            a[pos[:2]] = np.nan
            a[pos[2:]] = -np.nan if np.signbit(-np.nan) else np.copysign(np.nan, -1.0)
            for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                k = f(a, lib=lib)[0]
                assert np.isnan(k[:2]).all() and np.signbit(k[:2]).all(), f"{dt.__name__} n={n} head"
                assert np.isnan(k[-2:]).all() and not np.signbit(k[-2:]).any(), f"{dt.__name__} n={n} tail"
                mid = k[2:-2]
                assert (mid == np.sort(a[~np.isnan(a)])).all(), f"{dt.__name__} n={n} middle"


def pin_payload_64(lib):
    """A 64-bit payload (key + reference items) follows its key, all 64 bits."""
    rng = np.random.default_rng(RNG_SEED + 7)
    for dt in (np.uint64, np.int64, np.float64):
        for n in (2, 9, 16, 17, 100, 256):
            a = (_rand(dt, n, rng) if dt != np.float64 else _finite_floats(dt, n, rng))
            v = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
            order = np.argsort(a, kind="stable")
            for f in (oracle.insertion_sort, oracle.merge_sort, oracle.sort_one):
                k, vv = f(a, v, lib=lib)
                assert vv.dtype == np.uint64
                assert (k == a[order]).all() and (vv == v[order]).all(), f"{dt.__name__} n={n} {f.__name__}"
        off = np.array([0, 3, 3, 20, 21, 60], dtype=np.int32)
        a = _rand(np.uint64, 60, rng)
        v = rng.integers(0, 2**64, size=60, dtype=np.uint64, endpoint=False)
        k, vv = oracle.sort_segments(a, off, v, lib=lib)
        for i in range(off.size - 1):
            lo, hi = off[i], off[i + 1]
            order = np.argsort(a[lo:hi], kind="stable")
            assert (k[lo:hi] == a[lo:hi][order]).all() and (vv[lo:hi] == v[lo:hi][order]).all()


PINS = [pin_permutations, pin_small_words, pin_extremes, pin_random_vs_numpy,
        pin_payload_stable, pin_permutation_product, pin_fixed_stride, pin_segments,
        pin_float_vs_numpy, pin_float_signed_zeros_and_infinities, pin_float_nans_at_the_ends,
        pin_payload_64]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(oracle._get())


def test_threaded_driver_matches_serial():
    rng = np.random.default_rng(7)
    a = _rand(np.uint64, 1000 * 12, rng)
    assert (oracle.sort_fixed(a, 12, 1000, 12, threads=4) == oracle.sort_fixed(a, 12, 1000, 12)).all()
    off = np.concatenate([[0], np.cumsum(rng.integers(0, 60, size=500))]).astype(np.int32)
    b = _rand(np.int32, int(off[-1]), rng)
    k1, _ = oracle.sort_segments(b, off, threads=3)
    k2, _ = oracle.sort_segments(b, off)
    assert (k1 == k2).all()


# ------------------------------------------------------ planted mistakes --

MUTANTS = {
    # insertion sort: moves equal keys (breaks stability of the payload)
    "is_nonstrict": ("while (j > 0 && LT(k, keys[j - 1]))", "while (j > 0 && !LT(keys[j - 1], k))"),
    # insertion sort: never considers position 0
    "is_off_by_one": ("while (j > 0 && LT(k, keys[j - 1]))", "while (j > 1 && LT(k, keys[j - 1]))"),
    # merge: wrong comparison direction
    "merge_sign": ("if (LT(keys[b], keys[a]))", "if (LT(keys[a], keys[b]))"),
    # merge: drops the tail of the right run
    "merge_drop_tail": ("while (b < hi)  { tk[o] = keys[b];", "while (0)  { tk[o] = keys[b];"),
    # merge: payload taken from the wrong run
    "merge_payload": ("tk[o] = keys[b]; if (vals) tv[o] = vals[b]; ++b;",
                      "tk[o] = keys[b]; if (vals) tv[o] = vals[a]; ++b;"),
    # dispatcher: the insertion/merge threshold ignored (merge never used)...
    # ...and the fixed layout walking rows at the wrong pitch
    "fixed_pitch": ("keys + i * stride, NULL, n", "keys + i * n, NULL, n"),
    # segments: end taken from the wrong offset
    "segment_end": ("hi = offsets[i + 1];", "hi = offsets[i + 1] - 1;"),
    # unsigned keys compared as signed (an easy slip when stamping types)
    "u32_as_i32": ("ORACLE_DEFINE(uint32_t, u32, uint32_t, lt_u32)", "ORACLE_DEFINE(int32_t, u32, uint32_t, lt_i32)"),
    # floats: the native compare (signed zeros equal, NaNs unordered)
    "f32_native_compare": ("static inline int lt_f32(float a, float b) {",
                           "static inline int lt_f32(float a, float b) { return a < b;"),
    # floats: negatives ordered by ascending magnitude (raw sign-magnitude bits)
    "f64_negatives_unreversed": ("    if (sx != sy) return sx > sy;\n    return sx ? mx > my : mx < my;\n}\n\n/* One",
                                 "    if (sx != sy) return sx > sy;\n    return mx < my;\n}\n\n/* One"),
    # floats: positive before negative
    "f32_sign_order": ("    if (sx != sy) return sx > sy;      /* sign set first */",
                       "    if (sx != sy) return sx < sy;      /* sign set first */"),
    # the 64-bit payload stamped as a 32-bit one (payload halves lost)
    "v64_as_v32": ("ORACLE_DEFINE(uint64_t, u64_v64, uint64_t, lt_u64)",
                   "ORACLE_DEFINE(uint64_t, u64_v64, uint32_t, lt_u64)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTANTS[name]
    src = open(oracle_build.SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutant_src = tmp_path / "oracle_mutant.c"
    mutant_src.write_text(src.replace(old, new, 1))
    lib_path = str(tmp_path / "liboracle_mutant.so")
    oracle_build.build(src=str(mutant_src), out=lib_path)
    lib = oracle.load(lib_path)
    failed = []
    for pin in PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught the planted mistake {name}"
