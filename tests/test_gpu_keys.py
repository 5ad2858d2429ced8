"""Parity of the further key and item types with the CPU oracle: float and
double keys (IEEE 754 totalOrder) in every layout, and 64-bit keys with a
64-bit payload (the paper's key + reference items, Section 2.2).  Floats are
compared as bit patterns, so signed zeros and NaN payloads count."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, to_dev, tuned

pytestmark = pytest.mark.gpu

FLOATS = [np.float32, np.float64]
MODES = [ss.MODE_AUTO, ss.MODE_PERSISTENT, ss.MODE_PLAIN]
MODE_IDS = ["graph", "persistent", "plain"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield
    assert ss.device_status() == 0


def bits(a):
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def run_fixed(a, n, count, stride):
    t = to_dev(a)
    ss.sort_small(t, n, count=count, stride=stride)
    return from_dev(t)


def run_seg(keys, off, vals=None, mode=ss.MODE_AUTO):
    tk, to = to_dev(keys), to_dev(off)
    tv = to_dev(vals) if vals is not None else None
    ss.segmented_sort(tk, to, tv, mode=mode)
    return from_dev(tk), (from_dev(tv) if tv is not None else None)


@pytest.mark.parametrize("family", [0, 1, 2])
@pytest.mark.parametrize("dtype", FLOATS, ids=lambda d: np.dtype(d).name)
def test_float_keys_fixed_networks(dtype, family):
    count = 2 * 256 + 19
    with tuned(family=family):
        for n in range(2, 17):
            for seed, gen in ((n, inputs.float_keys), (n + 100, inputs.random_keys)):
                a = gen(dtype, n * count, seed)
                got = run_fixed(a, n, count, n)
                want = oracle.sort_fixed(a, n, count, n)
                assert (bits(got) == bits(want)).all(), f"n={n}: {first_mismatch(bits(got), bits(want), n)}"
        # the direct kernel (stride != n)
        a = inputs.float_keys(dtype, 13 * 300, 7)
        got = run_fixed(a, 12, 300, 13)
        assert (bits(got) == bits(oracle.sort_fixed(a, 12, 300, 13))).all()


@pytest.mark.parametrize("dtype", FLOATS, ids=lambda d: np.dtype(d).name)
def test_float_keys_fixed_rss(dtype):
    for n in (17, 33, 64, 65, 100, 128, 129, 200, 256):
        count = 41
        for seed, gen in ((n, inputs.float_keys), (n + 7, inputs.random_keys)):
            a = gen(dtype, n * count, seed)
            got = run_fixed(a, n, count, n)
            want = oracle.sort_fixed(a, n, count, n)
            assert (bits(got) == bits(want)).all(), f"n={n}: {first_mismatch(bits(got), bits(want), n)}"


def test_float_order_of_special_values():
    """-NaN < -inf < -1 < -0 < +0 < 1 < +inf < +NaN, checked on one array."""
    vals = np.array([np.nan, 1.0, -0.0, np.inf, 0.0, -1.0, -np.inf, np.copysign(np.nan, -1.0)],
                    dtype=np.float32)
    a = np.tile(vals, 64)
    got = run_fixed(a, 8, 64, 8).reshape(64, 8)
    for row in got:
        assert np.isnan(row[0]) and np.signbit(row[0])
        assert row[1] == -np.inf and row[2] == -1.0
        assert row[3] == 0.0 and np.signbit(row[3]) and row[4] == 0.0 and not np.signbit(row[4])
        assert row[5] == 1.0 and row[6] == np.inf and np.isnan(row[7]) and not np.signbit(row[7])


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dtype", FLOATS, ids=lambda d: np.dtype(d).name)
def test_float_keys_segmented(dtype, mode):
    rng = np.random.default_rng(3)
    sizes = np.concatenate([rng.integers(0, 257, size=1500), rng.integers(0, 17, size=2500)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    a = inputs.float_keys(dtype, total, 11)
    got, _ = run_seg(a, off, mode=mode)
    want, _ = oracle.sort_segments(a, off)
    assert (bits(got) == bits(want)).all(), first_mismatch(bits(got), bits(want))
    # distinct bit patterns are distinct keys under totalOrder: payloads are exact
    if dtype == np.float32:
        # an odd multiplier is a bijection modulo 2^32: distinct 32-bit patterns
        d = (np.random.default_rng(12).permutation(total).astype(np.uint64) * np.uint64(2654435761)
             + np.uint64(977)) & np.uint64(0xFFFFFFFF)
        d = d.astype(np.uint32)
    else:
        d = inputs.distinct_u64(total, seed=12)
    assert np.unique(d).size == total
    a = d.view(dtype)
    vals = inputs.segment_index_payload(off)
    gk, gv = run_seg(a, off, vals, mode=mode)
    wk, wv = oracle.sort_segments(a, off, vals)
    assert (bits(gk) == bits(wk)).all() and (gv == wv).all()
    assert ss.device_status() == 0


@pytest.mark.parametrize("family", [0, 1, 2])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_key_reference_pairs_64_64(mode, family):
    """uint64 keys with a uint64 reference, every size class, in every form."""
    sizes = inputs.geometric_sizes(20000, seed=51)
    sizes[:300] = np.arange(300) % 257
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = inputs.distinct_u64(total, seed=52)
    refs = inputs.splitmix64(53, total)  # arbitrary 64-bit references
    with tuned(family=family):
        gk, gv = run_seg(keys, off, refs, mode=mode)
    wk, wv = oracle.sort_segments(keys, off, refs)
    assert gv.dtype == np.uint64
    assert (gk == wk).all() and (gv == wv).all(), first_mismatch(gv, wv)
    assert ss.device_status() == 0


@pytest.mark.parametrize("dtype", [np.int64, np.float64], ids=lambda d: np.dtype(d).name)
def test_signed_and_float_keys_with_64bit_payload(dtype):
    sizes = inputs.geometric_sizes(8000, seed=61)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = inputs.distinct_u64(total, seed=62).view(dtype)
    refs = inputs.splitmix64(63, total)
    gk, gv = run_seg(keys, off, refs)
    wk, wv = oracle.sort_segments(keys, off, refs)
    assert (bits(gk) == bits(wk)).all() and (gv == wv).all()
    # duplicate keys: keys exact, (key, ref) pairs as a per-segment multiset
    k2 = inputs.random_keys(np.int64, total, seed=64).view(dtype).copy()
    k2[np.random.default_rng(1).random(total) < 0.4] = dtype(3)
    gk, gv = run_seg(k2, off, refs)
    wk, _ = oracle.sort_segments(k2, off, refs)
    assert (bits(gk) == bits(wk)).all()
    from helpers import pairs_multiset_equal
    assert pairs_multiset_equal(bits(gk), gv, bits(k2), refs, off) is None


def test_pairs_entry_point_and_payload_width_errors():
    import torch
    lib = ss.lib()
    keys, _, off = inputs.config4(nseg=3000, seed=71)
    refs = inputs.splitmix64(72, keys.size)
    tk, tr, to = to_dev(keys), to_dev(refs), to_dev(off)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.segmented_sort_pairs_u64(p(tk), p(tr), p(to), off.size - 1, stream) == 0
    wk, wv = oracle.sort_segments(keys, off, refs)
    assert (from_dev(tk) == wk).all() and (from_dev(tr) == wv).all()
    # 8-byte payloads need 64-bit keys; only 4 and 8 bytes exist
    k32 = to_dev(inputs.random_keys(np.uint32, keys.size, 3))
    assert lib.ss_segmented_sort_v(0, p(k32), p(tr), 8, p(to), off.size - 1, 0, stream) == -1
    assert lib.ss_segmented_sort_v(2, p(tk), p(tr), 2, p(to), off.size - 1, 0, stream) == -1
    assert lib.ss_segmented_sort_v(2, p(tk), ctypes.c_void_p(tr.data_ptr() + 4), 8, p(to), off.size - 1, 0,
                                   stream) == -2
