"""Comparator networks for n = 2..16 and the HIP code generator.

A network is a list of comparators ``(i, j)`` with ``i < j`` over channels
``0..n-1``; a comparator leaves the smaller value on channel ``i`` (paper,
Section 2.1).  *Size* is the comparator count, *depth* the number of levels of
independent comparators, counted as-soon-as-possible.

Sources (Section 2.2 collects best-known networks and generated ones):

* the size-optimal 10-channel network printed as Figure 2 (29 comparators);
* the best-known 16-channel network printed as Figure 3 (60 comparators);
* the recursive Bose-Nelson construction (Section 2.1, "split the input into
  first and second half, sort each, merge"), which reproduces Figure 1 and the
  locality-ordered Figure 4 comparator for comparator;
* windows of the printed networks: if the channels outside ``[r, r+m)`` carry
  -inf below and +inf above, every comparator crossing the window boundary
  never swaps, so the comparators inside the window form an m-channel sorting
  network.  Pruning Figures 2 and 3 gives smaller networks than Bose-Nelson
  for n = 9..16.

``best(n)`` picks the smallest network among these sources (then the
shallowest).  Every network is verified before emission with the 0-1
principle (a comparator network sorts every input iff it sorts all 2^n
inputs of zeros and ones), evaluated bit-parallel over all 2^n inputs.

``emit_header`` writes ``csrc/networks_gen.hpp``: one straight-line device
function per (family, n) that applies ``op(i, j)`` for each comparator, so
the compiler sees constant channel indices and keeps every channel in a VGPR.
"""
from __future__ import annotations

import os
import sys
from typing import List, Tuple

Network = List[Tuple[int, int]]

# Figure 2, channels renumbered from 0 (printed order).
FIG2_N10: Network = [(a - 1, b - 1) for a, b in [
    (5, 10), (4, 9), (3, 8), (2, 7), (1, 6), (2, 5), (7, 10), (1, 4), (6, 9), (1, 3),
    (4, 7), (8, 10), (1, 2), (3, 5), (6, 8), (9, 10), (2, 3), (5, 7), (8, 9), (4, 6),
    (3, 6), (7, 9), (2, 4), (5, 8), (3, 4), (7, 8), (4, 5), (6, 7), (5, 6)]]

# Figure 3, channels renumbered from 0 (printed order).
FIG3_N16: Network = [(a - 1, b - 1) for a, b in [
    (1, 2), (3, 4), (5, 6), (7, 8), (9, 10), (11, 12), (13, 14), (15, 16), (1, 3), (5, 7),
    (9, 11), (13, 15), (2, 4), (6, 8), (10, 12), (14, 16), (1, 5), (9, 13), (2, 6), (10, 14),
    (3, 7), (11, 15), (4, 8), (12, 16), (1, 9), (2, 10), (3, 11), (4, 12), (5, 13), (6, 14),
    (7, 15), (8, 16), (6, 11), (7, 10), (4, 13), (14, 15), (8, 12), (2, 3), (5, 9), (2, 5),
    (8, 14), (3, 9), (12, 15), (3, 5), (6, 7), (10, 11), (12, 14), (4, 9), (8, 13), (7, 9),
    (11, 13), (4, 6), (8, 10), (4, 5), (6, 7), (8, 9), (10, 11), (12, 13), (7, 8), (9, 10)]]

MAX_N = 16
FAMILIES = ("best", "bose_nelson")


# ------------------------------------------------------------ construction --

def bose_nelson(n: int) -> Network:
    """Bose-Nelson network for n channels in recursive (locality) order.

    sort(i, m) sorts channels [i, i+m): sort the first floor(m/2) channels,
    then the rest, then merge the two sorted runs.  merge(i, x, j, y) merges
    the sorted runs [i, i+x) and [j, j+y); its base cases are the 1+1, 1+2 and
    2+1 merges, and larger merges split both runs and merge three times.
    """
    out: Network = []

    def merge(i: int, x: int, j: int, y: int) -> None:
        if x == 1 and y == 1:
            out.append((i, j))
        elif x == 1 and y == 2:
            out.append((i, j + 1))
            out.append((i, j))
        elif x == 2 and y == 1:
            out.append((i, j))
            out.append((i + 1, j))
        else:
            assert x >= 1 and y >= 1, "unbalanced merge"
            a = x // 2
            b = y // 2 if x % 2 == 1 else (y + 1) // 2
            merge(i, a, j, b)
            merge(i + a, x - a, j + b, y - b)
            merge(i + a, x - a, j, b)

    def sort(i: int, m: int) -> None:
        if m < 2:
            return
        a = m // 2
        sort(i, a)
        sort(i + a, m - a)
        merge(i, a, i + a, m - a)

    sort(0, n)
    return out


def window(net: Network, lo: int, m: int) -> Network:
    """Comparators of ``net`` lying wholly inside channels [lo, lo+m), shifted to 0."""
    return [(i - lo, j - lo) for i, j in net if lo <= i and j < lo + m]


def best_window(net: Network, width: int, m: int) -> Network:
    """The window of size m of a width-channel network with fewest comparators."""
    cands = [window(net, lo, m) for lo in range(0, width - m + 1)]
    return min(cands, key=lambda w: (len(w), depth(w, m)))


def depth(net: Network, n: int) -> int:
    """Number of levels when each comparator is placed as early as possible."""
    ready = [0] * max(n, 1)
    d = 0
    for i, j in net:
        lvl = max(ready[i], ready[j]) + 1
        ready[i] = ready[j] = lvl
        d = max(d, lvl)
    return d


def levels(net: Network, n: int) -> List[Network]:
    """Group comparators into as-soon-as-possible levels (for reports)."""
    ready = [0] * max(n, 1)
    out: List[Network] = []
    for i, j in net:
        lvl = max(ready[i], ready[j])
        ready[i] = ready[j] = lvl + 1
        while len(out) <= lvl:
            out.append([])
        out[lvl].append((i, j))
    return out


def sorts_all_01(net: Network, n: int) -> bool:
    """0-1 principle check over all 2^n inputs, bit-parallel.

    Channel c is a 2^n-bit integer whose bit x is bit c of input x.  On zeros
    and ones a comparator's min is AND and its max is OR.  The output is
    sorted for every input iff no channel holds a 1 above a 0, i.e.
    out[c] & ~out[c+1] == 0 for all c.
    """
    if n < 2:
        return True
    nin = 1 << n
    full = (1 << nin) - 1
    ch = []
    for c in range(n):
        # bit x set iff (x >> c) & 1: a period of 2^(c+1) bits whose upper half is ones
        period = 1 << (c + 1)
        pattern = ((1 << (1 << c)) - 1) << (1 << c)
        span = period
        while span < nin:
            pattern |= pattern << span
            span *= 2
        ch.append(pattern & full)
    for i, j in net:
        if not (0 <= i < j < n):
            return False
        a, b = ch[i], ch[j]
        ch[i], ch[j] = a & b, a | b
    return all((ch[c] & ~ch[c + 1]) & full == 0 for c in range(n - 1))


def network(family: str, n: int) -> Network:
    """The network of a family for n channels (n <= 1: empty)."""
    if n < 2:
        return []
    if family == "bose_nelson":
        return bose_nelson(n)
    if family == "best":
        return best(n)
    raise ValueError(family)


def best(n: int) -> Network:
    """Fewest comparators among Bose-Nelson and the windows of Figures 2 and 3."""
    if n < 2:
        return []
    cands = [("bose_nelson", bose_nelson(n))]
    if n <= 16:
        cands.append(("fig3", FIG3_N16 if n == 16 else best_window(FIG3_N16, 16, n)))
    if n <= 10:
        cands.append(("fig2", FIG2_N10 if n == 10 else best_window(FIG2_N10, 10, n)))
    return min((c[1] for c in cands), key=lambda w: (len(w), depth(w, n)))


def table() -> List[dict]:
    rows = []
    for n in range(2, MAX_N + 1):
        row = {"n": n}
        for fam in FAMILIES:
            net = network(fam, n)
            row[fam] = (len(net), depth(net, n))
        rows.append(row)
    return rows


# ------------------------------------------------------------- emission --

HEADER_NAME = "networks_gen.hpp"


def render_header() -> str:
    lines = [
        "// Generated by paper_2002_05599_amd/networks.py -- do not edit by hand.",
        "// Comparator networks for 2..16 channels.  Family 0 = fewest comparators",
        "// (best-known lists of the paper's Figures 2 and 3 and their windows, or",
        "// Bose-Nelson where smaller); family 1 = Bose-Nelson (recursive construction).",
        "// Each run() applies op(i, j) for every comparator (i < j, min to i) in order.",
        "// Every list below passed the exhaustive 0-1 check when it was generated.",
        "#pragma once",
        "",
        "namespace ss {",
        "",
        "template <int Family, int N> struct Net;",
        "",
    ]
    for fi, fam in enumerate(FAMILIES):
        for n in range(0, MAX_N + 1):
            net = network(fam, n)
            if n >= 2 and not sorts_all_01(net, n):
                raise AssertionError(f"{fam} n={n} fails the 0-1 check")
            lines.append(f"template <> struct Net<{fi}, {n}> {{  // {fam}")
            lines.append(f"  static constexpr int kSize = {len(net)};")
            lines.append(f"  static constexpr int kDepth = {depth(net, n) if n >= 2 else 0};")
            lines.append("  template <class Op> __device__ __forceinline__ static void run(Op& op) {")
            if n < 2:
                lines.append("    (void)op;")
            else:
                # wrap long bodies over several lines
                chunks = [net[k:k + 8] for k in range(0, len(net), 8)]
                for ch in chunks:
                    lines.append("    " + " ".join(f"op({i}, {j});" for i, j in ch))
            lines.append("  }")
            lines.append("};")
            lines.append("")
    lines.append("}  // namespace ss")
    lines.append("")
    return "\n".join(lines)


def emit_header(path: str | None = None) -> str:
    if path is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", HEADER_NAME)
    text = render_header()
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)
    return path


if __name__ == "__main__":
    for r in table():
        print(r)
    print(emit_header(), file=sys.stderr)
