"""Parity of the device-wide sort (sample-sort partitions with the small
sorters as base case) with the CPU oracle: every key type, payloads, skewed
and duplicate-heavy inputs, sizes around every threshold (from about two
million keys a level partitions in two passes, by splitter block and then by
bucket; below, in one)."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, to_dev

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 17, 300, 4096, 4097, 10_001, 70_000, 1_000_003, 2_500_000, 9_000_001]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield
    assert ss.device_status() == 0


def bits(a):
    return a.view({4: np.uint32, 8: np.uint64}[a.dtype.itemsize])


def want_sorted(keys, vals=None):
    off = np.array([0, keys.size], dtype=np.int32)
    return oracle.sort_segments(keys, off, vals)


def run(keys, vals=None):
    tk = to_dev(keys)
    tv = to_dev(vals) if vals is not None else None
    ss.sort(tk, tv)
    return from_dev(tk), (from_dev(tv) if tv is not None else None)


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64],
                         ids=lambda d: np.dtype(d).name)
def test_device_sort_keys(dtype):
    for n in SIZES:
        a = inputs.float_keys(dtype, n, seed=n) if np.dtype(dtype).kind == "f" else inputs.random_keys(dtype, n, n)
        got, _ = run(a)
        want, _ = want_sorted(a)
        assert (bits(got) == bits(want)).all(), f"n={n}: {first_mismatch(bits(got), bits(want))}"


@pytest.mark.parametrize("n", [600_000, 4_000_000])
@pytest.mark.parametrize("kind", ["all_equal", "few", "zipf", "sorted", "reverse", "one_heavy", "narrow"])
def test_device_sort_skewed_inputs(kind, n):
    rng = np.random.default_rng(3)
    if kind == "all_equal":
        a = np.full(n, 77, np.uint32)
    elif kind == "few":
        a = rng.integers(0, 5, size=n).astype(np.uint32)
    elif kind == "zipf":
        a = inputs.zipf_keys(n, seed=4).astype(np.uint32)
    elif kind == "sorted":
        a = np.sort(inputs.random_keys(np.uint32, n, 5))
    elif kind == "reverse":
        a = np.sort(inputs.random_keys(np.uint32, n, 5))[::-1].copy()
    elif kind == "one_heavy":
        a = inputs.random_keys(np.uint32, n, 6)
        a[rng.random(n) < 0.7] = 123456
    else:  # values in a narrow band: many buckets of one value, many range buckets
        a = rng.integers(1000, 1000 + n // 12, size=n).astype(np.uint32)
    got, _ = run(a)
    want, _ = want_sorted(a)
    assert (got == want).all(), first_mismatch(got, want)


@pytest.mark.parametrize("vb", [4, 8])
def test_device_sort_payloads(vb):
    for n in (5000, 250_000, 3_000_000):
        keys = inputs.distinct_u64(n, seed=n + vb)
        vals = np.arange(n, dtype=np.uint32) if vb == 4 else inputs.splitmix64(9, n)
        gk, gv = run(keys, vals)
        wk, wv = want_sorted(keys, vals)
        assert (gk == wk).all() and (gv == wv).all()
    # duplicates with a payload: keys exact, pairs as a multiset
    for n in (300_000, 3_000_000):
        keys = inputs.random_keys(np.int64, n, 10)
        keys[np.random.default_rng(2).random(keys.size) < 0.5] = -3
        vals = np.arange(keys.size, dtype=np.uint32)
        gk, gv = run(keys, vals)
        wk, _ = want_sorted(keys, vals)
        assert (gk == wk).all()
        assert (np.sort(gv) == vals).all() and (keys[gv] == gk).all()


def test_device_sort_workspace_and_argument_errors():
    import torch
    lib = ss.lib()
    n = 100_000
    a = to_dev(inputs.random_keys(np.uint32, n, 1))
    need = ss.sort_workspace_bytes("uint32", n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.ss_sort(0, p(a), None, 0, n, p(ws), need - 1, stream) == -8
    assert lib.ss_sort(0, p(a), None, 4, n, p(ws), need, stream) == -1   # val_bytes without vals
    assert lib.ss_sort(0, p(a), p(a), 8, n, p(ws), need, stream) == -1   # 8-byte payload, 32-bit keys
    assert lib.ss_sort(9, p(a), None, 0, n, p(ws), need, stream) == -1
    # an unaligned workspace base is accepted when the size covers the alignment
    ws2 = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    assert lib.ss_sort(0, p(a), None, 0, n, ctypes.c_void_p(ws2.data_ptr() + 8), need + 248, stream) == 0
    got = from_dev(a)
    assert (got[1:] >= got[:-1]).all()
