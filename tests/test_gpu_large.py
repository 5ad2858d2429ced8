"""Parity of arrays and segments of 257..4096 keys (runs of 256 keys sorted by
Register Sample Sort, then merged in LDS by one work-group) with the CPU
oracle, in the fixed layout and the segmented forms, with payloads."""
import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, pairs_multiset_equal, to_dev, tuned

pytestmark = pytest.mark.gpu

SIZES = [257, 300, 511, 512, 513, 767, 1000, 1024, 2047, 2048, 3001, 4095, 4096]
MODES = [ss.MODE_AUTO, ss.MODE_PERSISTENT, ss.MODE_PLAIN]
MODE_IDS = ["graph", "persistent", "plain"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield
    assert ss.device_status() == 0


def run_fixed(a, n, count, stride):
    t = to_dev(a)
    ss.sort_small(t, n, count=count, stride=stride)
    return from_dev(t)


def run_seg(keys, off, vals=None, mode=ss.MODE_AUTO):
    tk, to = to_dev(keys), to_dev(off)
    tv = to_dev(vals) if vals is not None else None
    ss.segmented_sort(tk, to, tv, mode=mode)
    return from_dev(tk), (from_dev(tv) if tv is not None else None)


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64],
                         ids=lambda d: np.dtype(d).name)
def test_large_fixed(dtype):
    for n in SIZES:
        count = 5
        for k, dist in enumerate(("uniform", "few", "reverse")):
            if np.dtype(dtype).kind == "f":
                a = inputs.float_keys(dtype, n * count, seed=n + k) if dist == "uniform" else \
                    inputs.fixed_keys(np.int32, n, count, dist, seed=n + k).astype(dtype)
            else:
                a = inputs.fixed_keys(dtype, n, count, dist, seed=n + k)
            got = run_fixed(a, n, count, n)
            want = oracle.sort_fixed(a, n, count, n)
            bits = np.uint32 if a.dtype.itemsize == 4 else np.uint64
            assert (got.view(bits) == want.view(bits)).all(), f"n={n} {dist}: {first_mismatch(got, want, n)}"
    # a stride larger than n leaves the gap alone
    a = inputs.random_keys(dtype if np.dtype(dtype).kind != "f" else np.uint32, 700 * 3, seed=9)
    got = run_fixed(a, 600, 3, 700)
    assert (got == oracle.sort_fixed(a, 600, 3, 700)).all()


@pytest.mark.parametrize("family", [0, 1])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_large_segments_mixed_batch(mode, family):
    """Large segments among every other class, distinct 64-bit keys with 32- and
    64-bit payloads, and duplicate-heavy 32-bit keys."""
    rng = np.random.default_rng(5)
    sizes = np.concatenate([rng.integers(257, 4097, size=60), np.array(SIZES), rng.integers(0, 257, size=2000)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    with tuned(family=family):
        keys = inputs.distinct_u64(total, seed=6)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all() and (gv == wv).all(), first_mismatch(gv, wv)
        refs = inputs.splitmix64(7, total)
        gk, gr = run_seg(keys, off, refs, mode=mode)
        wk, wr = oracle.sort_segments(keys, off, refs)
        assert (gk == wk).all() and (gr == wr).all()
        k32 = inputs.random_keys(np.int32, total, seed=8)
        k32[rng.random(total) < 0.5] = 11
        v32 = inputs.segment_index_payload(off)
        gk, gv = run_seg(k32, off, v32, mode=mode)
        wk, _ = oracle.sort_segments(k32, off, v32)
        assert (gk == wk).all(), first_mismatch(gk, wk)
        assert pairs_multiset_equal(gk, gv, k32, v32, off) is None
    assert ss.device_status() == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64], ids=lambda d: np.dtype(d).name)
def test_large_segments_largest_key_ties(dtype):
    """Merge shares at the end of a run pair hold slots past both runs; with many
    keys equal to the type's largest value (one segment made only of them),
    such a slot never takes the place of a real key or its payload."""
    rng = np.random.default_rng(14)
    sizes = np.array([257, 300, 513, 777, 1025, 1500, 2049, 3001, 4095, 4096, 259, 20, 0, 600])
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    top = np.iinfo(dtype).max
    keys = inputs.random_keys(dtype, total, seed=15)
    keys[rng.random(total) < 0.3] = top
    keys[off[5]:off[6]] = top
    v32 = inputs.segment_index_payload(off)
    payloads = [v32] + ([inputs.splitmix64(16, total)] if keys.itemsize == 8 else [])
    want, _ = oracle.sort_segments(keys, off, v32)
    for mode in MODES:
        for vals in payloads:
            gk, gv = run_seg(keys, off, vals, mode=mode)
            assert (gk == want).all(), (mode, first_mismatch(gk, want))
            assert pairs_multiset_equal(gk, gv, keys, vals, off) is None, mode
    assert ss.device_status() == 0


def test_large_segments_other_knobs():
    """Insertion sort in place of RSS (IS+SN), insertion-sort run finishing, a
    level cap of 1 and a first level of 4 buckets, on large segments."""
    rng = np.random.default_rng(9)
    sizes = np.concatenate([rng.integers(257, 4097, size=12), rng.integers(0, 300, size=200)])
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = inputs.distinct_u64(total, seed=10)
    vals = inputs.segment_index_payload(off)
    wk, wv = oracle.sort_segments(keys, off, vals)
    for knobs in ({"large_sort": 1}, {"family": 2}, {"rss_level_cap": 1}, {"rss_k_large": 4}, {"rss_finish": 1}):
        with tuned(**knobs):
            for mode in (ss.MODE_AUTO, ss.MODE_PLAIN):
                gk, gv = run_seg(keys, off, vals, mode=mode)
                assert (gk == wk).all() and (gv == wv).all(), (knobs, mode)
        n = 1500
        a = inputs.random_keys(np.int64, n * 3, seed=11)
        a[rng.random(a.size) < 0.3] = -1
        with tuned(**knobs):
            got = run_fixed(a, n, 3, n)
        assert (got == oracle.sort_fixed(a, n, 3, n)).all(), knobs


def test_large_segments_noalloc_entry():
    """The no-allocation entry point carries the large class too."""
    import ctypes
    import torch
    rng = np.random.default_rng(12)
    sizes = np.concatenate([rng.integers(257, 4097, size=20), rng.integers(0, 100, size=500)])
    off = inputs.offsets_from_sizes(sizes)
    keys = inputs.random_keys(np.uint32, int(off[-1]), seed=13)
    tk, to = to_dev(keys), to_dev(off)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = ss.lib().ss_segmented_sort_noalloc(0, ctypes.c_void_p(tk.data_ptr()), None, ctypes.c_void_p(to.data_ptr()),
                                            off.size - 1, stream)
    assert st == 0
    want, _ = oracle.sort_segments(keys, off)
    assert (from_dev(tk) == want).all()
