"""Parity of the segmented (CSR, ragged) sorts with the CPU oracle, in all three modes."""
import numpy as np
import pytest

import oracle
import paper_2002_05599_amd as ss
from paper_2002_05599_amd import inputs
from helpers import first_mismatch, from_dev, pairs_multiset_equal, to_dev

pytestmark = pytest.mark.gpu

TYPES = [np.uint32, np.int32, np.uint64, np.int64]
MODES = [ss.MODE_AUTO, ss.MODE_PERSISTENT, ss.MODE_PLAIN]
MODE_IDS = ["graph", "persistent", "plain"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ss.lib()
    yield


def run_seg(keys, off, vals=None, mode=ss.MODE_AUTO):
    tk = to_dev(keys)
    to = to_dev(off)
    tv = to_dev(vals) if vals is not None else None
    ss.segmented_sort(tk, to, tv, mode=mode)
    return from_dev(tk), (from_dev(tv) if tv is not None else None)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
def test_mixed_sizes_keys_only(dtype, mode):
    rng = np.random.default_rng(5)
    sizes = np.concatenate([np.arange(0, 257), rng.integers(0, 257, size=700), rng.integers(0, 17, size=900)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes) + 3  # offsets need not start at 0
    keys = inputs.random_keys(dtype, int(off[-1]) + 5, seed=21)
    got, _ = run_seg(keys, off, mode=mode)
    want, _ = oracle.sort_segments(keys, off)
    assert (got == want).all(), first_mismatch(got, want)
    assert ss.device_status() == 0


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
def test_payload_distinct_keys_exact(dtype, mode):
    sizes = inputs.geometric_sizes(6000, seed=8)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = inputs.distinct_u64(total, seed=8)
    if np.dtype(dtype).itemsize == 4:
        # distinct 32-bit keys: a permutation of a random distinct set
        keys = (np.random.default_rng(8).permutation(np.arange(total, dtype=np.int64) * 7919 + 13)
                & 0xFFFFFFFF).astype(np.uint32)
        assert np.unique(keys).size == total
    keys = keys.view(dtype) if keys.dtype.itemsize == np.dtype(dtype).itemsize else keys.astype(dtype)
    vals = inputs.segment_index_payload(off)
    gk, gv = run_seg(keys, off, vals, mode=mode)
    wk, wv = oracle.sort_segments(keys, off, vals)
    assert (gk == wk).all(), first_mismatch(gk, wk)
    assert (gv == wv).all(), first_mismatch(gv, wv)


@pytest.mark.parametrize("dtype", [np.uint32, np.int64], ids=lambda d: np.dtype(d).name)
def test_payload_duplicate_keys_multiset(dtype):
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 257, size=1500)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    keys = rng.integers(0, 5, size=total).astype(dtype)
    info = np.iinfo(dtype)
    keys[rng.random(total) < 0.1] = info.max  # collides with the padding value
    vals = np.arange(total, dtype=np.uint32)
    gk, gv = run_seg(keys, off, vals)
    wk, wv = oracle.sort_segments(keys, off, vals)
    assert (gk == wk).all()
    bad = pairs_multiset_equal(gk, gv, keys, vals, off)
    assert bad is None, f"segment {bad}: payload is not a permutation of its pairs"


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_config3_shape_small(dist):
    keys, off = inputs.config3(nseg=4000, dist=dist, seed=3)
    for mode in MODES:
        got, _ = run_seg(keys, off, mode=mode)
        want, _ = oracle.sort_segments(keys, off)
        assert (got == want).all(), (mode, first_mismatch(got, want))


def test_config4_shape_small_all_modes_agree():
    keys, vals, off = inputs.config4(nseg=30000, seed=4)
    wk, wv = oracle.sort_segments(keys, off, vals)
    for mode in MODES:
        gk, gv = run_seg(keys, off, vals, mode=mode)
        assert (gk == wk).all() and (gv == wv).all(), mode


def test_oversize_and_bad_offsets_flagged():
    sizes = np.array([5, 4097, 20, 0, 1, 256, 300])
    off = inputs.offsets_from_sizes(sizes)
    keys = inputs.random_keys(np.uint32, int(off[-1]), seed=1)
    got, _ = run_seg(keys, off)
    assert ss.device_status() == -3
    assert ss.device_status() == 0  # reading clears it
    want, _ = oracle.sort_segments(keys, off)
    lo, hi = off[1], off[2]
    assert (got[lo:hi] == keys[lo:hi]).all(), "oversize segment must be left untouched"
    mask = np.ones(keys.size, bool)
    mask[lo:hi] = False
    assert (got[mask] == want[mask]).all()
    # decreasing offsets
    off2 = np.array([0, 10, 4, 30], dtype=np.int32)
    keys2 = inputs.random_keys(np.uint32, 30, seed=2)
    run_seg(keys2, off2)
    assert ss.device_status() == -1


def test_empty_and_trivial_batches():
    assert ss.device_status() == 0
    got, _ = run_seg(np.arange(10, dtype=np.uint32)[::-1].copy(), np.array([0], dtype=np.int32))
    assert (got == np.arange(10)[::-1]).all()
    got, _ = run_seg(np.array([3, 1, 2], dtype=np.int64), np.array([0, 1, 2, 3], dtype=np.int32))
    assert (got == [3, 1, 2]).all()


def test_graph_replays_with_changing_inputs():
    """The cached graph is replayed with new buffers, sizes and shapes; eager work in between."""
    import torch
    for rep in range(5):
        nseg = [1000, 1000, 4000, 10, 2500][rep]
        keys, vals, off = inputs.config4(nseg=nseg, seed=40 + rep)
        tk, tv, to = to_dev(keys), to_dev(vals), to_dev(off)
        ss.segmented_sort(tk, to, tv, mode=ss.MODE_AUTO)
        scratch = torch.ones(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        del scratch
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (from_dev(tk) == wk).all() and (from_dev(tv) == wv).all(), rep


def test_repeat_runs_identical():
    keys, off = inputs.config3(nseg=3000, dist="zipf", seed=12)
    r1, _ = run_seg(keys, off)
    r2, _ = run_seg(keys, off)
    assert (r1 == r2).all()


def _check_sampled(got_k, keys, off, got_v=None, vals=None, nsample=4000):
    rng = np.random.default_rng(0)
    nseg = off.size - 1
    segs = np.unique(np.concatenate([rng.integers(0, nseg, size=nsample), [0, nseg - 1]]))
    for i in segs:
        lo, hi = int(off[i]), int(off[i + 1])
        wk, wv = oracle.sort_one(keys[lo:hi], None if vals is None else vals[lo:hi])
        assert (got_k[lo:hi] == wk).all(), f"segment {i}"
        if vals is not None:
            assert (got_v[lo:hi] == wv).all(), f"segment {i} payload"


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_config3_full_size_sampled(dist):
    """2^20 CSR arrays of 17..256 int32 keys: sampled segments vs the oracle + invariants."""
    keys, off = inputs.config3(dist=dist)
    got, _ = run_seg(keys, off)
    assert ss.device_status() == 0
    _check_sampled(got, keys, off)
    # every segment sorted; multiset fingerprint per batch
    d = got[1:].astype(np.int64) - got[:-1].astype(np.int64)
    boundary = np.zeros(got.size - 1, bool)
    boundary[off[1:-1] - 1] = True
    assert ((d >= 0) | boundary).all()
    assert np.sort(got, kind="stable").tobytes() == np.sort(keys, kind="stable").tobytes()


@pytest.mark.slow
def test_config4_full_size_sampled():
    """10^7 ragged segments, u64 distinct keys + u32 payload (the bench batch)."""
    keys, vals, off = inputs.config4()
    gk, gv = run_seg(keys, off, vals)
    assert ss.device_status() == 0
    _check_sampled(gk, keys, off, gv, vals)
    # payload is the in-segment index: it must index the original segment
    seg_start = np.repeat(off[:-1], np.diff(off)).astype(np.int64)
    assert (keys[seg_start + gv.astype(np.int64)] == gk).all()


@pytest.mark.parametrize("k", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("mode", [ss.MODE_AUTO, ss.MODE_PLAIN], ids=["graph", "plain"])
def test_first_level_bucket_counts_with_payload(k, mode):
    """Every first-level bucket count on the RSS classes, distinct 64-bit keys
    with payload (exact) and duplicate-heavy 32-bit keys (keys exact)."""
    from helpers import tuned
    with tuned(rss_k_small=min(k, 16), rss_k_mid=min(k, 32), rss_k_large=min(k, 64)):
        sizes = np.random.default_rng(k).integers(17, 257, size=3000)
        off = inputs.offsets_from_sizes(sizes)
        total = int(off[-1])
        keys = inputs.distinct_u64(total, seed=k)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all(), first_mismatch(gk, wk)
        assert (gv == wv).all(), first_mismatch(gv, wv)
        dup = (inputs.random_keys(np.uint32, total, seed=k) % 5).astype(np.uint32)
        gk, _ = run_seg(dup, off, mode=mode)
        wk, _ = oracle.sort_segments(dup, off)
        assert (gk == wk).all(), first_mismatch(gk, wk)
        assert ss.device_status() == 0


@pytest.mark.parametrize("mode", [ss.MODE_AUTO, ss.MODE_PERSISTENT], ids=["graph", "persistent"])
@pytest.mark.parametrize("dtype", TYPES, ids=lambda d: np.dtype(d).name)
def test_mixed_size_network_tiles(dtype, mode):
    """net_mix = 1: segments of 2..16 keys sorted in batch order with the
    network of each wave's largest segment (max padding), with and without
    payload, next to RSS segments and empty/size-1 segments."""
    old = ss.get_tuning("net_mix")
    ss.set_tuning("net_mix", 1)
    try:
        rng = np.random.default_rng(11)
        sizes = np.concatenate([rng.integers(0, 17, size=5000), rng.integers(17, 257, size=300),
                                np.arange(0, 17)])
        rng.shuffle(sizes)
        off = inputs.offsets_from_sizes(sizes)
        total = int(off[-1])
        # keys only, duplicate-heavy and extreme values included
        keys = inputs.random_keys(dtype, total, seed=12)
        info = np.iinfo(dtype)
        keys[rng.random(total) < 0.2] = info.max
        keys[rng.random(total) < 0.1] = info.min
        got, _ = run_seg(keys, off, mode=mode)
        want, _ = oracle.sort_segments(keys, off)
        assert (got == want).all(), first_mismatch(got, want)
        # payload with distinct keys: exact
        dk = inputs.distinct_u64(total, seed=13)
        dk = dk.view(dtype) if np.dtype(dtype).itemsize == 8 else \
            (np.random.default_rng(13).permutation(total).astype(np.int64) * 7 + 3).astype(dtype)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(dk, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(dk, off, vals)
        assert (gk == wk).all(), first_mismatch(gk, wk)
        assert (gv == wv).all(), first_mismatch(gv, wv)
        assert ss.device_status() == 0
    finally:
        ss.set_tuning("net_mix", old)


def test_graph_replays_back_to_back_without_sync():
    """Several calls of the cached graph queued on one stream, each on its own
    buffers with its own segment count, with no host synchronisation between
    them (as the bench issues them): every output must match the oracle."""
    import torch
    cases = []
    for rep, nseg in enumerate([3000, 800, 12000, 5, 4000, 1]):
        keys, vals, off = inputs.config4(nseg=nseg, seed=60 + rep)
        cases.append((keys, vals, off, to_dev(keys), to_dev(vals), to_dev(off)))
    torch.cuda.synchronize()
    for _, _, _, tk, tv, to in cases:
        ss.segmented_sort(tk, to, tv, mode=ss.MODE_AUTO)
    torch.cuda.synchronize()
    for rep, (keys, vals, off, tk, tv, _) in enumerate(cases):
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (tk.cpu().numpy() == wk).all() and (tv.cpu().numpy() == wv).all(), rep
    assert ss.device_status() == 0


KERNEL_FORMS = [dict(persist_split=s, interleave=i, net_mix=m) for s in (0, 1) for i in (0, 1) for m in (0, 1)
                if not (s == 1 and i == 1)]  # interleaving only applies to the single kernel


@pytest.mark.parametrize("form", KERNEL_FORMS,
                         ids=lambda f: f"split{f['persist_split']}-il{f['interleave']}-mix{f['net_mix']}")
@pytest.mark.parametrize("mode", [ss.MODE_AUTO, ss.MODE_PERSISTENT], ids=["graph", "persistent"])
def test_persistent_kernel_forms(form, mode):
    """Every persistent kernel layout the autotuner may choose: one kernel for all
    classes (with and without interleaving) or one per kind, per-size or mixed
    network tiles.  Mixed sizes with RSS segments, keys-only duplicates and
    distinct 64-bit keys with payload."""
    from helpers import tuned
    rng = np.random.default_rng(17)
    sizes = np.concatenate([rng.integers(0, 257, size=2500), rng.integers(0, 17, size=6000),
                            rng.integers(17, 65, size=1500)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    with tuned(**form):
        for dtype in (np.uint32, np.int64):
            keys = inputs.random_keys(dtype, total, seed=18)
            keys[rng.random(total) < 0.3] = 7
            got, _ = run_seg(keys, off, mode=mode)
            want, _ = oracle.sort_segments(keys, off)
            assert (got == want).all(), (dtype, first_mismatch(got, want))
        keys = inputs.distinct_u64(total, seed=19)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all() and (gv == wv).all()
        assert ss.device_status() == 0


@pytest.mark.parametrize("family", [0, 1, 2])
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_network_families_segmented(family, mode):
    """Both network families and insertion sort (family 2) in the segmented
    network tiles and RSS finishing."""
    from helpers import tuned
    with tuned(family=family):
        sizes = inputs.geometric_sizes(20000, seed=21)
        off = inputs.offsets_from_sizes(sizes)
        total = int(off[-1])
        keys = inputs.distinct_u64(total, seed=22)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all() and (gv == wv).all()
        k32 = inputs.random_keys(np.int32, total, seed=23)
        got, _ = run_seg(k32, off, mode=mode)
        want, _ = oracle.sort_segments(k32, off)
        assert (got == want).all(), first_mismatch(got, want)


def test_workspace_grows_while_another_stream_runs():
    """Stream A's working memory grows (stream-ordered) while a large batch on
    stream B is still in flight: both results must match the oracle."""
    import torch
    sa = torch.cuda.Stream()
    sb = torch.cuda.Stream()
    kb, vb, ob = inputs.config4(nseg=400_000, seed=31)
    tb = (to_dev(kb), to_dev(vb), to_dev(ob))
    small = inputs.config4(nseg=100, seed=32)
    big = inputs.config4(nseg=300_000, seed=33)
    ta_small = tuple(to_dev(x) for x in small)
    ta_big = tuple(to_dev(x) for x in big)
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        ss.segmented_sort(ta_small[0], ta_small[2], ta_small[1])  # A's workspace sized for 100 segments
    with torch.cuda.stream(sb):
        ss.segmented_sort(tb[0], tb[2], tb[1])                    # B busy with a large batch
    with torch.cuda.stream(sa):
        ss.segmented_sort(ta_big[0], ta_big[2], ta_big[1])        # A grows while B runs
    torch.cuda.synchronize()
    for (k, v, o), (tk, tv, _) in ((small, ta_small), (big, ta_big), ((kb, vb, ob), tb)):
        wk, wv = oracle.sort_segments(k, o, v)
        assert (tk.cpu().numpy() == wk).all() and (tv.cpu().numpy() == wv).all()
    assert ss.device_status() == 0


def test_stream_copy_probe():
    """The bandwidth probe copies bytes exactly and rejects misaligned sizes."""
    import torch
    src = torch.from_numpy(inputs.random_keys(np.uint32, (1 << 20) + 64, seed=3)).cuda()
    dst = torch.zeros_like(src)
    ss.stream_copy(dst, src)
    assert torch.equal(dst, src)
    with pytest.raises(ss.SmallSortError):
        ss.stream_copy(dst[1:], src[1:])


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_insertion_sort_above_16_segmented(mode):
    """The IS+SN hybrid (large_sort=1): segments of 17..256 keys sorted by
    insertion sort, 2..16 by networks; mixed sizes, payload, duplicates."""
    from helpers import tuned
    rng = np.random.default_rng(41)
    sizes = np.concatenate([rng.integers(0, 257, size=3000), rng.integers(0, 17, size=2000)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    with tuned(large_sort=1):
        keys = inputs.distinct_u64(total, seed=42)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all() and (gv == wv).all()
        k32 = inputs.random_keys(np.int32, total, seed=43)
        k32[rng.random(total) < 0.3] = -5
        got, _ = run_seg(k32, off, mode=mode)
        want, _ = oracle.sort_segments(k32, off)
        assert (got == want).all(), first_mismatch(got, want)
        assert ss.device_status() == 0


MAPPINGS = [dict(rss_bound_tiny=16, rss_bound_small=16, rss_bound_mid=64),
            dict(rss_bound_tiny=16, rss_bound_small=32, rss_bound_mid=96),
            dict(rss_bound_tiny=16, rss_bound_small=48, rss_bound_mid=128),
            dict(rss_bound_tiny=16, rss_bound_small=64, rss_bound_mid=64),
            dict(rss_bound_tiny=32, rss_bound_small=64, rss_bound_mid=128),
            dict(rss_bound_tiny=24, rss_bound_small=40, rss_bound_mid=128),
            dict(rss_bound_tiny=32, rss_bound_small=32, rss_bound_mid=32),
            dict(rss_oversample=1), dict(rss_oversample=4), dict(rss_finish=0), dict(rss_finish=1),
            dict(rss_finish=1, rss_bound_tiny=16, rss_bound_small=16, rss_bound_mid=64),
            dict(rss_finish=1, rss_bound_tiny=32, rss_bound_small=64, rss_bound_mid=128),
            dict(rss_finish=0, rss_bound_tiny=32, rss_oversample=4)]


@pytest.mark.parametrize("knobs", MAPPINGS, ids=lambda k: "-".join(f"{a}{b}" for a, b in k.items()))
@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_lane_group_mappings_and_oversampling(knobs, mode):
    """The tuned wave-to-segment mapping (which RSS lane group takes which sizes)
    and the oversampling of the 4-bucket levels, in every segmented form:
    distinct 64-bit keys with payload and duplicate-heavy 32-bit keys."""
    from helpers import tuned
    rng = np.random.default_rng(91)
    sizes = np.concatenate([np.arange(0, 257), rng.integers(17, 129, size=3000), rng.integers(0, 257, size=2000)])
    rng.shuffle(sizes)
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    with tuned(**knobs):
        keys = inputs.distinct_u64(total, seed=92)
        vals = inputs.segment_index_payload(off)
        gk, gv = run_seg(keys, off, vals, mode=mode)
        wk, wv = oracle.sort_segments(keys, off, vals)
        assert (gk == wk).all() and (gv == wv).all()
        dup = (inputs.random_keys(np.uint32, total, seed=93) % 7).astype(np.uint32)
        gk, _ = run_seg(dup, off, mode=mode)
        wk, _ = oracle.sort_segments(dup, off)
        assert (gk == wk).all(), first_mismatch(gk, wk)
        assert ss.device_status() == 0
