"""Parity of Register Sample Sort (n = 17..256, fixed layout) with the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, to_dev

pytestmark = pytest.mark.gpu

TYPES = [np.uint32, np.int32, np.uint64, np.int64]
SIZES = [17, 18, 24, 31, 32, 33, 47, 63, 64, 65, 96, 127, 128, 129, 160, 200, 255, 256]


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


def special(dtype, n, count, kind, seed):
    info = np.iinfo(dtype)
    rng = np.random.default_rng(seed)
    if kind == "all_equal":
        return np.full(n * count, 12345, dtype=dtype)
    if kind == "two_values":
        return np.where(rng.random(n * count) < 0.5, 7, 9).astype(dtype)
    if kind == "max_heavy":
        a = inputs.random_keys(dtype, n * count, seed)
        a[rng.random(n * count) < 0.4] = info.max
        a[rng.random(n * count) < 0.1] = info.min
        return a
    if kind == "zipf":
        return inputs.zipf_keys(n * count, seed).astype(dtype)
    if kind == "organ":
        row = np.concatenate([np.arange(n // 2), np.arange(n - n // 2)[::-1]]).astype(dtype)
        return np.tile(row, count)
    if kind == "one_big_dup":
        a = inputs.random_keys(dtype, n * count, seed)
        a[rng.random(n * count) < 0.8] = 42
        return a
    raise ValueError(kind)


@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", SIZES)
def test_rss_distributions(n, dtype):
    count = 4 * 16 + 5  # several work-groups and a ragged tail at every group size
    for k, dist in enumerate(inputs.DISTRIBUTIONS):
        a = inputs.fixed_keys(dtype, n, count, dist, seed=1000 + 13 * n + k)
        got = run_fixed(a, n, count, n)
        want = oracle.sort_fixed(a, n, count, n)
        assert (got == want).all(), f"{dist}: {first_mismatch(got, want, n)}"


@pytest.mark.parametrize("kind", ["all_equal", "two_values", "max_heavy", "zipf", "organ", "one_big_dup"])
@pytest.mark.parametrize("dtype", [np.uint32, np.int64], ids=lambda d: np.dtype(d).name)
def test_rss_duplicates_and_extremes(kind, dtype):
    for n in (17, 40, 64, 100, 128, 256):
        count = 37
        a = special(dtype, n, count, kind, seed=n)
        got = run_fixed(a, n, count, n)
        want = oracle.sort_fixed(a, n, count, n)
        assert (got == want).all(), f"{kind} n={n}: {first_mismatch(got, want, n)}"


def test_rss_every_size_u32():
    """Every n in 17..256 once (u32, uniform)."""
    for n in range(17, 257):
        count = 9
        a = inputs.random_keys(np.uint32, n * count, seed=n * 7)
        got = run_fixed(a, n, count, n)
        want = oracle.sort_fixed(a, n, count, n)
        assert (got == want).all(), f"n={n}: {first_mismatch(got, want, n)}"


TUNINGS = [dict(rss_k_small=4), dict(rss_k_small=8), dict(rss_k_small=16),
           dict(rss_k_mid=4), dict(rss_k_mid=8), dict(rss_k_mid=16), dict(rss_k_mid=32),
           dict(rss_k_large=4), dict(rss_k_large=8), dict(rss_k_large=16), dict(rss_k_large=32),
           dict(rss_k_large=64), dict(family=0), dict(family=1), dict(family=2), dict(large_sort=1),
           dict(rss_oversample=1), dict(rss_oversample=2), dict(rss_oversample=4),
           dict(rss_bound_tiny=16, rss_bound_small=16), dict(rss_bound_tiny=16, rss_bound_small=32),
           dict(rss_bound_tiny=16, rss_bound_small=48), dict(rss_bound_mid=96), dict(rss_bound_mid=64),
           dict(rss_finish=1), dict(rss_bound_tiny=32), dict(rss_bound_tiny=24),
           dict(rss_bound_tiny=32, family=2), dict(rss_bound_tiny=32, rss_finish=1),
           dict(rss_bound_tiny=32, rss_oversample=4), dict(rss_bound_tiny=16)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "-".join(f"{k}={v}" for k, v in t.items()))
def test_rss_tuning_variants(tuning):
    """Every first-level bucket count and family (2: buckets finished by
    insertion sort), and insertion sort in place of RSS (large_sort=1, the
    IS+SN hybrid), the lane-group mappings (8-lane groups up to 16..32 keys)
    and bucket finishes: uniform keys of every class, duplicate-heavy keys
    (three-way splits) and 64-bit keys."""
    from helpers import tuned
    with tuned(**tuning):
        for n in (17, 20, 24, 32, 33, 48, 64, 65, 100, 128, 129, 200, 256):
            a = inputs.random_keys(np.int32, n * 50, seed=n)
            got = run_fixed(a, n, 50, n)
            assert (got == oracle.sort_fixed(a, n, 50, n)).all(), (tuning, n)
            for kind in ("zipf", "two_values", "one_big_dup", "max_heavy"):
                a = special(np.uint64, n, 21, kind, seed=n + 1)
                got = run_fixed(a, n, 21, n)
                want = oracle.sort_fixed(a, n, 21, n)
                assert (got == want).all(), (tuning, n, kind, first_mismatch(got, want, n))


def test_rss_stride_and_repeat():
    n, stride, count = 100, 130, 77
    a = inputs.random_keys(np.uint64, stride * count, seed=4)
    got = run_fixed(a, n, count, stride)
    assert (got == oracle.sort_fixed(a, n, count, stride)).all()
    assert (run_fixed(a, n, count, stride) == got).all()


@pytest.mark.parametrize("tiny", [16, 32])
@pytest.mark.parametrize("finish", [0, 1])
@pytest.mark.parametrize("cap", [1, 2])
@pytest.mark.parametrize("kind", ["uniform", "zipf", "two_values", "max_heavy", "one_big_dup"])
def test_rss_level_cap_fallback_fixed(cap, kind, finish, tiny):
    """Register Sample Sort stopped after `cap` levels: every bucket still above
    16 keys goes through the rank-counting fallback.  With a first level of 4
    buckets, arrays of 65..256 keys always leave such buckets, so the fallback
    runs on every array of those sizes; with both bucket finishes (the
    rank-counting finish must leave the fallback's buckets in place)."""
    from helpers import tuned
    with tuned(rss_level_cap=cap, rss_k_small=4, rss_k_mid=4, rss_k_large=4, rss_finish=finish, rss_bound_tiny=tiny):
        for dtype in (np.uint32, np.int64):
            for n in (17, 24, 32, 40, 64, 100, 128, 200, 256):
                count = 37
                if kind == "uniform":
                    a = inputs.fixed_keys(dtype, n, count, "uniform", seed=3 * n + cap)
                else:
                    a = special(dtype, n, count, kind, seed=n + cap)
                got = run_fixed(a, n, count, n)
                want = oracle.sort_fixed(a, n, count, n)
                assert (got == want).all(), (cap, kind, n, first_mismatch(got, want, n))


@pytest.mark.parametrize("finish", [0, 1])
@pytest.mark.parametrize("cap", [1, 2])
@pytest.mark.parametrize("mode", [ss.MODE_AUTO, ss.MODE_PLAIN], ids=["graph", "plain"])
def test_rss_level_cap_fallback_segmented_payload(cap, mode, finish):
    """The fallback carries payloads: distinct keys (payload exact) and
    duplicate-heavy keys (keys exact, payload a per-segment permutation), with
    both first-level widths (narrow forces the fallback, wide rarely needs it)."""
    from helpers import pairs_multiset_equal, tuned
    sizes = np.random.default_rng(cap).integers(17, 257, size=1500)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    for k in (4, 16):
        with tuned(rss_level_cap=cap, rss_k_small=k, rss_k_mid=k, rss_k_large=k, rss_finish=finish):
            keys = inputs.distinct_u64(total, seed=cap + k)
            vals = inputs.segment_index_payload(off)
            tk, tv, to = to_dev(keys), to_dev(vals), to_dev(off)
            ss.segmented_sort(tk, to, tv, mode=mode)
            gk, gv = from_dev(tk), from_dev(tv)
            wk, wv = oracle.sort_segments(keys, off, vals)
            assert (gk == wk).all(), first_mismatch(gk, wk)
            assert (gv == wv).all(), first_mismatch(gv, wv)
            dup = (inputs.random_keys(np.uint32, total, seed=k) % 3).astype(np.uint32)
            dup[np.random.default_rng(k).random(total) < 0.2] = np.iinfo(np.uint32).max
            vals = np.arange(total, dtype=np.uint32)
            tk, tv = to_dev(dup), to_dev(vals)
            ss.segmented_sort(tk, to, tv, mode=mode)
            gk, gv = from_dev(tk), from_dev(tv)
            wk, _ = oracle.sort_segments(dup, off)
            assert (gk == wk).all(), first_mismatch(gk, wk)
            assert pairs_multiset_equal(gk, gv, dup, vals, off) is None
