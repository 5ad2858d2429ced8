"""Comparator networks: exhaustive 0-1 checks and pins to the paper's figures (no GPU).

The 0-1 principle (a network sorts every input iff it sorts every 0/1 input)
is evaluated here with numpy over all 2^n inputs, independently of the
bit-parallel checker inside the generator.
"""
import os
import re

import numpy as np
import pytest

from paper_2002_05599_amd import networks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    """Comparators from a figure fixture, renumbered from 0."""
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = map(int, line.split())
        out.append((a - 1, b - 1))
    return out


def sorts_01_numpy(net, n):
    if n < 2:
        return True
    x = ((np.arange(1 << n, dtype=np.uint32)[:, None] >> np.arange(n, dtype=np.uint32)) & 1).astype(np.uint8)
    for i, j in net:
        lo = np.minimum(x[:, i], x[:, j])
        hi = np.maximum(x[:, i], x[:, j])
        x[:, i], x[:, j] = lo, hi
    return bool((x[:, 1:] >= x[:, :-1]).all())


def asap_dag(net, n):
    """Each comparator keyed by its channels and its ASAP level; order-free."""
    ready = [0] * n
    out = []
    for i, j in net:
        lvl = max(ready[i], ready[j])
        ready[i] = ready[j] = lvl + 1
        out.append((lvl, i, j))
    return sorted(out)


@pytest.mark.parametrize("family", networks.FAMILIES)
@pytest.mark.parametrize("n", range(2, 17))
def test_every_emitted_network_sorts(family, n):
    net = networks.network(family, n)
    assert all(0 <= i < j < n for i, j in net)
    assert sorts_01_numpy(net, n)
    assert networks.sorts_all_01(net, n)


def test_checker_rejects_broken_networks():
    net = networks.network("best", 12)
    for drop in (0, len(net) // 2, len(net) - 1):
        broken = net[:drop] + net[drop + 1:]
        assert not sorts_01_numpy(broken, 12)
        assert not networks.sorts_all_01(broken, 12)


def test_figures_transcribed():
    assert networks.FIG2_N10 == load_golden("fig2_optimal_size_10.txt")
    assert networks.FIG3_N16 == load_golden("fig3_best_16.txt")


def test_bose_nelson_reproduces_figures_1_and_4():
    assert networks.bose_nelson(6) == load_golden("fig1_bose_nelson_6.txt")
    assert networks.bose_nelson(16) == load_golden("fig4_bose_nelson_locality_16.txt")


def test_figure_5_is_figure_4_reordered():
    f4 = load_golden("fig4_bose_nelson_locality_16.txt")
    f5 = load_golden("fig5_bose_nelson_parallel_16.txt")
    assert asap_dag(f4, 16) == asap_dag(f5, 16)
    assert sorts_01_numpy(f5, 16)


def test_printed_sizes_and_depths():
    # Section 2.1: ten channels, optimal size 29 with nine levels.
    assert (len(networks.FIG2_N10), networks.depth(networks.FIG2_N10, 10)) == (29, 9)
    assert (len(networks.FIG3_N16), networks.depth(networks.FIG3_N16, 16)) == (60, 10)
    f1 = load_golden("fig1_bose_nelson_6.txt")
    assert len(f1) == 12
    assert len(load_golden("fig4_bose_nelson_locality_16.txt")) == 65


def test_windows_of_printed_networks_sort():
    for net, width in ((networks.FIG2_N10, 10), (networks.FIG3_N16, 16)):
        for m in range(2, width):
            for lo in range(0, width - m + 1):
                assert sorts_01_numpy(networks.window(net, lo, m), m), (width, lo, m)


def test_best_sizes():
    # smallest of Bose-Nelson and the windows of Figures 2 and 3
    want = {2: 1, 3: 3, 4: 5, 5: 9, 6: 12, 7: 16, 8: 19, 9: 25, 10: 29, 11: 36,
            12: 40, 13: 46, 14: 51, 15: 56, 16: 60}
    for n, size in want.items():
        assert len(networks.best(n)) == size
        assert len(networks.best(n)) <= len(networks.bose_nelson(n))
    # Section 2.2: best and Bose-Nelson agree in size for n <= 8
    for n in range(2, 9):
        assert len(networks.best(n)) == len(networks.bose_nelson(n))


def test_emitted_header_matches_lists():
    path = os.path.join(os.path.dirname(networks.__file__), "csrc", networks.HEADER_NAME)
    text = open(path).read()
    assert text == networks.render_header(), "networks_gen.hpp is stale; rerun networks.py"
    blocks = re.findall(r"struct Net<(\d+), (\d+)> \{.*?run\(Op& op\) \{(.*?)\n  \}", text, re.S)
    assert len(blocks) == 2 * 17
    for fam, n, body in blocks:
        n = int(n)
        net = [(int(a), int(b)) for a, b in re.findall(r"op\((\d+), (\d+)\)", body)]
        assert net == networks.network(networks.FAMILIES[int(fam)], n)
        assert sorts_01_numpy(net, n)
