"""The no-allocation segmented entry point (ss_segmented_sort_noalloc), called
through the C ABI, against the allocating entry point (ss_segmented_sort) on
the same inputs: bit-exact keys and payloads, two calls in a row with the
second one smaller, plus the host-side rejection of a batch beyond the fixed
scratch."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, to_dev

pytestmark = pytest.mark.gpu

SS_ESCRATCH = -7


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _call(entry, code, tk, tv, to, *extra):
    import torch
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return entry(code, _ptr(tk), _ptr(tv), _ptr(to), to.numel() - 1, *extra, stream)


def _both(keys, off, vals, code):
    """(noalloc result, allocating result) on fresh device copies of the input."""
    import torch
    lib = ss.lib()
    a = [to_dev(keys), to_dev(vals) if vals is not None else None, to_dev(off)]
    b = [to_dev(keys), to_dev(vals) if vals is not None else None, to_dev(off)]
    assert _call(lib.ss_segmented_sort_noalloc, code, *a) == 0
    assert _call(lib.ss_segmented_sort, code, *b, ss.MODE_PERSISTENT) == 0
    torch.cuda.synchronize()
    out = []
    for k, v, _ in (a, b):
        out.append((k.cpu().numpy(), v.cpu().numpy() if v is not None else None))
    return out


def _check_pair(keys, off, vals, code):
    (nk, nv), (ak, av) = _both(keys, off, vals, code)
    assert (nk == ak).all(), first_mismatch(nk, ak)
    if vals is not None:
        assert (nv == av).all(), first_mismatch(nv, av)
    wk, wv = oracle.sort_segments(keys, off, vals)
    assert (nk == wk).all(), first_mismatch(nk, wk)
    if vals is not None:
        assert (nv == wv).all(), first_mismatch(nv, wv)


def test_noalloc_matches_allocating_entry_two_calls_second_smaller():
    # call 1: ragged batch, distinct uint64 keys with payload (every size class)
    keys, vals, off = inputs.config4(nseg=60_000, seed=71)
    _check_pair(keys, off, vals, ss.KEY_CODES["uint64"])
    # call 2, smaller, on the same scratch: mixed sizes, int32 keys only, with
    # offsets that do not start at 0 and empty segments
    rng = np.random.default_rng(72)
    sizes = np.concatenate([np.arange(0, 257), rng.integers(0, 17, size=900), rng.integers(17, 257, size=300)])
    rng.shuffle(sizes)
    off2 = inputs.offsets_from_sizes(sizes) + 5
    keys2 = inputs.random_keys(np.int32, int(off2[-1]) + 3, seed=73)
    _check_pair(keys2, off2, None, ss.KEY_CODES["int32"])
    assert ss.device_status() == 0


def test_noalloc_back_to_back_on_one_stream():
    """Calls ordered on one stream with no host sync between them: each one
    rebuilds the scratch contents it uses, so every result is exact."""
    import torch
    lib = ss.lib()
    cases = []
    for rep, nseg in enumerate([20_000, 3_000, 500]):
        k, v, o = inputs.config4(nseg=nseg, seed=80 + rep)
        cases.append((k, v, o, to_dev(k), to_dev(v), to_dev(o)))
    torch.cuda.synchronize()
    for _, _, _, tk, tv, to in cases:
        assert _call(lib.ss_segmented_sort_noalloc, ss.KEY_CODES["int64"], tk, tv, to) == 0
    torch.cuda.synchronize()
    for k, v, o, tk, tv, _ in cases:
        wk, wv = oracle.sort_segments(k.view(np.int64), o, v)
        assert (tk.cpu().numpy().view(np.int64) == wk).all()
        assert (tv.cpu().numpy() == wv).all()


def test_noalloc_rejects_batch_beyond_scratch():
    import torch
    lib = ss.lib()
    tk = torch.zeros(16, dtype=torch.int32, device="cuda").view(torch.uint32)
    to = torch.zeros(16, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.ss_segmented_sort_noalloc(0, _ptr(tk), None, _ptr(to), ss.NOALLOC_MAX_SEGMENTS + 1, stream)
    assert st == SS_ESCRATCH
    assert b"no-allocation" in lib.ss_strerror(st)
    assert lib.ss_segmented_sort_noalloc(0, _ptr(tk), None, _ptr(to), 0, stream) == 0
    assert lib.ss_segmented_sort_noalloc(9, _ptr(tk), None, _ptr(to), 3, stream) == -1
