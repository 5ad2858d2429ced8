"""Autotuner for the library's variant choices (run on the GPU).

Knobs (see include/smallsort.h): network family; first-level bucket count of
Register Sample Sort per size class; the most rounds of lane groups per RSS
tile, one persistent kernel per kind or one for all, tile interleaving (single
kernel) and work-groups per CU of the persistent ragged kernels.  The paper
found the best variant and RSS parameters to differ from machine to machine
(Sections 4.2 and 4.5); here they are measured on the GPU at hand.

Workloads: fixed-size arrays of 4..16 keys (family); one CSR batch per RSS
size class (its bucket count); for the segmented-sort knobs the sum of the
10^7-segment ragged batch with payload and the 2^20-array RSS-only batch, at
the sizes the benchmark uses (a quarter of each with --quick).

Method: coordinate descent.  For each knob in turn every allowed value is
timed on a representative workload with the other knobs fixed, and the
fastest is kept if it beats the current value by more than 1% (otherwise the
current value stays).  A measurement is the median over ``reps`` calls, each on a
fresh copy of the input (restored outside the timed region) and bracketed by
HIP events on the calling stream.

The result is a flat JSON object ({"knob": value, ..., "arch": ..., "rocm":
...}) that ``ss_load_tuning`` reads; the binding loads
``tuning_<arch>.json`` next to the library automatically when its arch and
ROCm version match the running system.  A separate report records every
measurement.

    python -m paper_2002_05599_amd.autotune [--quick] [--out PATH] [--report PATH]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def system_tag():
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return arch, str(torch.version.hip)


def default_path(arch=None):
    return os.path.join(HERE, f"tuning_{arch or 'gfx950'}.json")


def _timer(fn, restore, reps):
    import torch
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        restore()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


class Workloads:
    """Representative inputs, resident on the device, with pristine copies."""

    def __init__(self, quick=False):
        import torch
        from . import inputs
        scale = 4 if quick else 1
        # fixed-size arrays for the network family (u32 and u64)
        self.fixed = []
        for dt in (np.uint32, np.uint64):
            for n in (4, 8, 12, 16):
                a = torch.from_numpy(inputs.fixed_keys(dt, n, (1 << 22) // scale, "uniform", seed=n)).cuda()
                self.fixed.append((n, a, a.clone()))
        # RSS classes: CSR batches with sizes inside each class
        self.rss = {}
        for knob, lo, hi in (("rss_k_small", 17, 64), ("rss_k_mid", 65, 128), ("rss_k_large", 129, 256)):
            off = inputs.offsets_from_sizes(inputs.csr_sizes((1 << 18) // scale, lo, hi, seed=hi))
            k = torch.from_numpy(inputs.random_keys(np.uint64, int(off[-1]), seed=lo)).cuda()
            self.rss[knob] = (k, k.clone(), torch.from_numpy(off).cuda())
        # ragged batch of the 10^7-segment benchmark (a quarter with --quick)
        k, v, off = inputs.config4(nseg=10_000_000 // scale, seed=44)
        self.ragged = (torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(off).cuda())
        self.ragged_src = tuple(t.clone() for t in self.ragged[:2])
        # RSS-only batch of the 2^20-array benchmark: int32 arrays of 17..256 keys
        k, off = inputs.config3(nseg=(1 << 20) // scale, dist="uniform", seed=7)
        k = torch.from_numpy(k).cuda()
        self.rss_all = (k, k.clone(), torch.from_numpy(off).cuda())
        torch.cuda.synchronize()

    def time_family(self, reps):
        """The family shapes the fixed-size sorts and every network inside RSS."""
        from . import sort_small
        total = 0.0
        for n, a, src in self.fixed:
            total += _timer(lambda: sort_small(a, n), lambda: a.copy_(src), reps)
        for knob in self.rss:
            total += self.time_rss(knob, reps)
        return total

    def time_rss(self, knob, reps):
        from . import segmented_sort
        k, src, off = self.rss[knob]
        return _timer(lambda: segmented_sort(k, off), lambda: k.copy_(src), reps)

    def time_ragged_only(self, reps, mode=0):
        from . import segmented_sort
        k, v, off = self.ragged

        def restore():
            k.copy_(self.ragged_src[0])
            v.copy_(self.ragged_src[1])

        return _timer(lambda: segmented_sort(k, off, v, mode=mode), restore, reps)

    def time_rss_all(self, reps, mode=0):
        from . import segmented_sort
        k, src, off = self.rss_all
        return _timer(lambda: segmented_sort(k, off, mode=mode), lambda: k.copy_(src), reps)

    def time_ragged(self, reps, mode=0):
        """Objective of the segmented-sort knobs: ragged batch + RSS-only batch."""
        return self.time_ragged_only(reps, mode) + self.time_rss_all(reps, mode)


NOISE = 0.01

SPACE = [
    ("family", [0, 1], "family"),
    ("rss_k_small", [4, 8, 16], "rss"),
    ("rss_k_mid", [4, 8, 16, 32], "rss"),
    ("rss_k_large", [4, 8, 16, 32, 64], "rss"),
    ("rss_rounds", [4, 8, 16, 32, 64], "ragged"),
    ("persist_split", [0, 1], "ragged"),
    ("net_mix", [0, 1], "ragged"),
    ("interleave", [0, 1], "ragged"),
    ("persist_occ", [0, 1, 2, 3], "ragged"),
]


def tune(quick=False, reps=5, log=print):
    from . import get_tuning, set_tuning
    w = Workloads(quick=quick)
    best = {name: get_tuning(name) for name, _, _ in SPACE}
    report = {}
    for name, values, kind in SPACE:
        results = {}
        for v in values:
            set_tuning(name, v)
            if kind == "family":
                ms = w.time_family(reps)
            elif kind == "rss":
                ms = w.time_rss(name, reps)
            else:
                ms = w.time_ragged(reps)
            results[v] = ms
            log(f"  {name}={v}: {ms:.4f} ms")
        # keep the current value unless another is faster by more than the noise
        # threshold (1%)
        choice = min(results, key=results.get)
        if best[name] in results and results[choice] > (1.0 - NOISE) * results[best[name]]:
            choice = best[name]
        set_tuning(name, choice)
        best[name] = choice
        report[name] = {"ms": {str(k): v for k, v in results.items()}, "best": choice}
        log(f"{name} -> {choice}")
    # tuned persistent graph form vs one launch per size class
    for mode, name in ((0, "graph"), (2, "plain")):
        report[f"ragged_{name}_ms"] = w.time_ragged_only(reps, mode)
        report[f"rss_{name}_ms"] = w.time_rss_all(reps, mode)
    return best, report


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--quick", action="store_true", help="smaller workloads")
    p.add_argument("--reps", type=int, default=5)
    p.add_argument("--out", default=None)
    p.add_argument("--report", default=None)
    args = p.parse_args()
    import torch
    assert torch.cuda.is_available(), "the autotuner runs on the GPU"
    arch, rocm = system_tag()
    t0 = time.time()
    best, report = tune(quick=args.quick, reps=args.reps, log=lambda s: print(s, flush=True))
    print(json.dumps({k: v for k, v in report.items() if k.endswith("_ms")}), flush=True)
    out = args.out or default_path(arch)
    doc = dict(best)
    doc.update({"arch": arch, "rocm": rocm})
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"arch": arch, "rocm": rocm, "seconds": time.time() - t0, "best": best,
                       "measurements": report}, f, indent=1)
    print(json.dumps(doc), file=sys.stderr)


if __name__ == "__main__":
    main()
