"""Parity of the fixed-layout sorts (networks, n = 2..16) with the CPU oracle.

All inputs are seeded; every comparison is bit-exact.
"""
import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, to_dev, tuned

pytestmark = pytest.mark.gpu

TYPES = [np.uint32, np.int32, np.uint64, np.int64]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield
    assert ss.device_status() == 0


def run_fixed(keys_np, n, count, stride):
    t = to_dev(keys_np)
    ss.sort_small(t, n, count=count, stride=stride)
    return from_dev(t)


FAMILIES = [0, 1, 2]  # fewest comparators, Bose-Nelson, insertion sort


@pytest.mark.parametrize("family", FAMILIES, ids=lambda f: f"family{f}")
@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", range(2, 17))
def test_networks_match_oracle_all_distributions(n, dtype, family):
    # several 256-array tiles plus a ragged tail
    count = 3 * 256 + 37
    with tuned(family=family):
        for k, dist in enumerate(inputs.DISTRIBUTIONS):
            a = inputs.fixed_keys(dtype, n, count, dist, seed=100 + 7 * n + k)
            got = run_fixed(a, n, count, n)
            want = oracle.sort_fixed(a, n, count, n)
            assert (got == want).all(), f"{dist}: {first_mismatch(got, want, n)}"
        # the direct (unstaged) kernel: a stride other than n
        a = inputs.fixed_keys(dtype, n, 300, "uniform", seed=n)
        a = np.concatenate([a.reshape(300, n), a.reshape(300, n)[:, :1]], axis=1).reshape(-1)
        got = run_fixed(a, n, 300, n + 1)
        assert (got == oracle.sort_fixed(a, n, 300, n + 1)).all()


@pytest.mark.parametrize("family", FAMILIES, ids=lambda f: f"family{f}")
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.int32], ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", range(2, 17))
def test_zero_one_principle_on_device(n, dtype, family):
    """Every 0/1 input of length n (2^n arrays) comes out sorted (0-1 principle)."""
    x = np.arange(1 << n, dtype=np.uint64)
    bits = ((x[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)
    info = np.iinfo(dtype)
    lo, hi = (info.min, info.max)  # the extremes stand for 0 and 1
    a = np.where(bits == 1, hi, lo).astype(dtype).reshape(-1)
    with tuned(family=family):
        got = run_fixed(a, n, 1 << n, n).reshape(-1, n)
    ones = bits.sum(axis=1)
    want = np.where(np.arange(n)[None, :] >= (n - ones)[:, None], hi, lo).astype(dtype)
    assert (got == want).all()


@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n,stride", [(5, 8), (16, 17), (3, 3), (12, 40)])
def test_stride_gap_untouched(n, stride, dtype):
    count = 600
    a = inputs.random_keys(dtype, count * stride, seed=stride * 31 + n)
    got = run_fixed(a, n, count, stride)
    want = oracle.sort_fixed(a, n, count, stride)
    assert (got == want).all(), first_mismatch(got, want, stride)


@pytest.mark.parametrize("dtype", [np.uint32, np.int64], ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", [4, 7, 16])
def test_unaligned_base_pointer(n, dtype):
    import torch
    count = 700
    a = inputs.random_keys(dtype, count * n + 1, seed=77 + n)
    t = to_dev(a)
    ss.sort_small(t[1:], n, count=count, stride=n)  # base offset by one key: not 16-byte aligned
    got = from_dev(t)
    want = a.copy()
    want[1:] = oracle.sort_fixed(a[1:], n, count, n)
    assert (got == want).all()
    del torch


@pytest.mark.parametrize("count", [1, 2, 255, 256, 257, 511, 513])
def test_tile_boundaries(count):
    for n in (8, 13, 16):
        a = inputs.random_keys(np.uint32, count * n, seed=count + n)
        got = run_fixed(a, n, count, n)
        assert (got == oracle.sort_fixed(a, n, count, n)).all(), (n, count)


def test_noop_sizes_leave_data():
    a = inputs.random_keys(np.uint64, 100, seed=5)
    for n, count in ((0, 10), (1, 100), (8, 0)):
        got = run_fixed(a, n, count, max(n, 1))
        assert (got == a).all()


def test_extremes_and_duplicates_signed():
    for dt in (np.int32, np.int64):
        info = np.iinfo(dt)
        vals = np.array([info.min, info.min + 1, -1, 0, 1, info.max - 1, info.max], dtype=dt)
        rng = np.random.default_rng(3)
        for n in (2, 9, 16):
            a = vals[rng.integers(0, vals.size, size=n * 1000)]
            got = run_fixed(a, n, 1000, n)
            assert (got == oracle.sort_fixed(a, n, 1000, n)).all()


def test_repeat_runs_identical():
    a = inputs.random_keys(np.uint64, 16 * 5000, seed=11)
    r1 = run_fixed(a, 16, 5000, 16)
    r2 = run_fixed(a, 16, 5000, 16)
    assert (r1 == r2).all()


def _row_invariants(before, after, n):
    """Rows sorted, and per-row sum and xor unchanged (multiset fingerprints)."""
    b = before.reshape(-1, n)
    g = after.reshape(-1, n)
    assert (g[:, 1:] >= g[:, :-1]).all(), "a row is not sorted"
    bu = b.view(np.uint64 if b.itemsize == 8 else np.uint32).astype(np.uint64)
    gu = g.view(np.uint64 if g.itemsize == 8 else np.uint32).astype(np.uint64)
    with np.errstate(over="ignore"):
        assert (bu.sum(axis=1) == gu.sum(axis=1)).all()
    assert (np.bitwise_xor.reduce(bu, axis=1) == np.bitwise_xor.reduce(gu, axis=1)).all()


@pytest.mark.slow
@pytest.mark.parametrize("dtype,n", [(np.uint32, 16), (np.int64, 16), (np.uint32, 8), (np.uint32, 5)],
                         ids=["u32-16", "i64-16", "u32-8", "u32-5"])
def test_full_size_sampled(dtype, n):
    """2^24 arrays (the bench workload): sampled rows vs the oracle, all rows by invariants."""
    count = 1 << 24
    a = inputs.fixed_keys(dtype, n, count, "uniform", seed=2)
    got = run_fixed(a, n, count, n)
    rng = np.random.default_rng(0)
    rows = np.unique(rng.integers(0, count, size=20000))
    rows = np.concatenate([rows, [0, count - 1]])
    sub_in = a.reshape(count, n)[rows].reshape(-1)
    want = oracle.sort_fixed(sub_in, n, rows.size, n)
    assert (got.reshape(count, n)[rows].reshape(-1) == want).all()
    _row_invariants(a, got, n)


def test_config1_exact():
    """100,000 arrays of 8 uint32 keys, seed 1: every row vs the oracle."""
    a = inputs.config1()
    got = run_fixed(a, 8, 100_000, 8)
    want = oracle.sort_fixed(a, 8, 100_000, 8)
    assert (got == want).all(), first_mismatch(got, want, 8)


@pytest.mark.parametrize("apt,half,wide,wider", [(1, 0, 0, 0), (2, 0, 0, 0), (4, 0, 0, 0), (1, 0x1FFFC, 0, 0),
                                                 (1, 0x0AAA8, 0, 0), (2, 0x1FFFC, 0, 0), (1, 0, 0x1FFFC, 0),
                                                 (1, 0x1FFFC, 0x15554, 0), (2, 0, 0x1FFFC, 0), (1, 0, 0, 0x1FFFC),
                                                 (1, 0x0AAA8, 0x15554, 0x0CCCC)],
                         ids=["apt1", "apt2", "apt4", "apt1-half", "apt1-half-odd", "apt2-half", "apt1-wide",
                              "apt1-wide-even-half-odd", "apt2-wide", "apt1-wider", "apt1-mixed"])
@pytest.mark.parametrize("dtype", [np.uint32, np.int64, np.float32], ids=lambda d: np.dtype(d).name)
def test_arrays_per_thread(apt, half, wide, wider, dtype):
    """Tiles of 1, 2 or 4 arrays per thread (reduced where the tile would not
    fit), and, where one array per thread is used, tiles staged by 128-thread
    work-groups or by 512- or 1024-thread work-groups over 256 arrays, for
    every n or mixed across n: several tiles and a ragged tail for every n."""
    with tuned(fixed_apt=apt, fixed_half=half, fixed_wide=wide, fixed_wider=wider):
        for n in range(2, 17):
            count = 3 * 1024 + 77
            a = (inputs.float_keys(dtype, n * count, seed=n) if np.dtype(dtype).kind == "f"
                 else inputs.fixed_keys(dtype, n, count, "uniform", seed=n))
            got = run_fixed(a, n, count, n)
            want = oracle.sort_fixed(a, n, count, n)
            bits = np.uint32 if a.dtype.itemsize == 4 else np.uint64
            assert (got.view(bits) == want.view(bits)).all(), f"n={n}: {first_mismatch(got, want, n)}"
