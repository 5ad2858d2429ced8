"""Seeded workload generators (no GPU)."""
import numpy as np

from paper_2002_05599_amd import inputs


def test_splitmix64_reference_vector():
    # First outputs of SplitMix64 from state 0 (the generator's published test vector).
    got = [int(x) for x in inputs.splitmix64(0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_deterministic_and_offsettable():
    a = inputs.splitmix64(9, 100)
    assert (a == inputs.splitmix64(9, 100)).all()
    assert (a[40:] == inputs.splitmix64(9, 60, start=40)).all()


def test_distributions_shapes():
    for dist in inputs.DISTRIBUTIONS:
        for dt in (np.uint32, np.int64):
            k = inputs.fixed_keys(dt, 7, 50, dist, seed=2)
            assert k.dtype == dt and k.size == 350
            rows = k.reshape(50, 7)
            if dist == "few":
                assert rows.min() >= 0 and rows.max() <= 3
            if dist == "sorted":
                assert (rows[:, 1:] >= rows[:, :-1]).all()
            if dist == "reverse":
                assert (rows[:, 1:] <= rows[:, :-1]).all()


def test_geometric_sizes():
    s = inputs.geometric_sizes(200_000, seed=4)
    assert s.min() >= 1 and s.max() <= 256
    assert abs(s.mean() - 24.0) < 0.5


def test_distinct_keys_and_payload():
    k, v, off = inputs.config4(nseg=20_000, seed=4)
    assert np.unique(k).size == k.size
    for i in (0, 1, 777, 19_999):
        lo, hi = off[i], off[i + 1]
        assert (v[lo:hi] == np.arange(hi - lo)).all()


def test_zipf_range():
    z = inputs.zipf_keys(100_000, seed=3)
    assert z.min() >= 1 and z.dtype == np.int32
    assert (z == 1).mean() > 0.05  # heavy head
