"""Autotuner for the library's variant choices (run on the GPU).

The paper found the best network variant and the best Register Sample Sort
parameters to differ from machine to machine (Sections 4.2 and 4.5); here
they are measured on the GPU at hand, separately for 32-bit and 64-bit keys.

Per key width (workloads of that width; 64-bit keys carry a uint32 payload):
  family           network family or insertion sort (fixed arrays of 4..16 keys
                   plus the RSS batches, whose buckets the networks finish;
                   for 64-bit keys also the ragged batch)
  fixed_apt        arrays per thread of the fixed-layout kernels (items per
                   thread; fixed arrays of 2..16 keys: it applies wherever the
                   tile of several arrays per thread fits)
  fixed_half, fixed_wide, fixed_wider
                   per n = 2..16, whether the one-array-per-thread tile of
                   arrays of n keys is staged by 256 threads, by 128, or by
                   512 or 1024 threads over 256 arrays (each n tuned on its
                   own fixed batch of that n, back-to-back calls, the forms
                   alternating)
  rss_bound_tiny, rss_bound_small, rss_bound_mid
                   the wave-to-segment mapping: which segment sizes get 8, 16,
                   32 or 64 lanes (CSR batches of 17..256, 17..64 and 65..128
                   keys, and a ragged batch of geometric sizes, mean 24: for
                   64-bit keys the 10^7-segment batch of the global knobs)
  rss_k_small/mid/large
                   first-level bucket count of each lane-group class (a CSR
                   batch of sizes within the class)
  rss_oversample   oversampling a of the 4-bucket levels (the RSS batch)
  rss_finish       RSS buckets finished by networks or by rank counting (the
                   RSS batch)
For every width together (the ragged 10^7-segment batch plus the 2^20-array
RSS batch): rss_rounds, persist_split, net_mix, interleave, persist_occ.

Method: coordinate descent.  For each knob every allowed value is timed with
the others fixed (median of ``reps`` calls, each on a fresh copy of the input
restored outside the timed region, bracketed by HIP events on the calling
stream); the fastest replaces the current value only if it is faster by more
than 1%.  Every candidate's output is compared, bit for bit, with the output
of the library's default settings on the same input (sorting has one correct
result: keys always, payloads where keys are distinct); a candidate that
differs is rejected and reported.

The result is a flat JSON object ({"u32.family": 1, ..., "rss_rounds": 64,
"arch": ..., "rocm": ...}) that ``ss_load_tuning`` reads; the binding loads
``tuning_<arch>.json`` next to the library automatically when its arch and
ROCm version match.  The report records every measurement in ms and GB/s.

    python -m paper_2002_05599_amd.autotune [--quick] [--out PATH] [--report PATH]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

PER_WIDTH = ("family", "fixed_apt", "fixed_half", "rss_bound_tiny", "rss_bound_small", "rss_bound_mid", "rss_k_small", "rss_k_mid",
             "rss_k_large", "rss_oversample", "rss_finish")
GLOBAL = ("rss_rounds", "persist_split", "net_mix", "interleave", "persist_occ")
NOISE = 0.01


def system_tag():
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return arch, str(torch.version.hip)


def default_path(arch=None):
    return os.path.join(HERE, f"tuning_{arch or 'gfx950'}.json")


class Case:
    """One timed input: device buffers, pristine copies, the call that sorts
    them, the bytes it must move, and the reference output."""

    def __init__(self, name, call, bufs, nbytes):
        self.name = name
        self.call = call            # call(bufs) sorts bufs in place
        self.bufs = bufs            # device tensors sorted in place
        self.src = [b.clone() for b in bufs]
        self.nbytes = nbytes
        self.ref = None

    def restore(self):
        for b, s in zip(self.bufs, self.src):
            b.copy_(s)

    def time(self, reps):
        """Median event time of one call (ms); the last call's output stays in bufs."""
        import torch
        stream = torch.cuda.current_stream()
        times = []
        for _ in range(reps):
            self.restore()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            self.call(self.bufs)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times))

    def record_reference(self):
        import torch
        self.restore()
        self.call(self.bufs)
        torch.cuda.synchronize()
        self.ref = [b.clone() for b in self.bufs]

    def output_matches(self):
        import torch
        torch.cuda.synchronize()
        return all(torch.equal(b.view(torch.uint8), r.view(torch.uint8)) for b, r in zip(self.bufs, self.ref))


def _fixed_case(width, n, count, seed):
    import torch
    from . import inputs, sort_small
    dt = np.uint32 if width == "u32" else np.uint64
    a = torch.from_numpy(inputs.fixed_keys(dt, n, count, "uniform", seed=seed)).cuda()
    return Case(f"{width} fixed n={n}", lambda b: sort_small(b[0], n), [a], 2 * a.numel() * a.element_size())


def _csr_case(width, nseg, lo, hi, seed, sizes=None, what=None):
    import torch
    from . import inputs, segmented_sort
    if sizes is None:
        sizes = inputs.csr_sizes(nseg, lo, hi, seed=seed)
    what = what or f"CSR {lo}..{hi}"
    off = inputs.offsets_from_sizes(sizes)
    total = int(off[-1])
    to = torch.from_numpy(off).cuda()
    if width == "u32":
        k = torch.from_numpy(inputs.random_keys(np.uint32, total, seed=lo)).cuda()
        return Case(f"u32 {what}", lambda b: segmented_sort(b[0], to), [k], 8 * total + 4 * nseg)
    k = torch.from_numpy(inputs.distinct_u64(total, seed=lo)).cuda()
    v = torch.from_numpy(inputs.segment_index_payload(off)).cuda()
    return Case(f"u64+payload {what}", lambda b: segmented_sort(b[0], to, b[1]), [k, v],
                24 * total + 4 * nseg)


class Workloads:
    """Representative inputs per key width, resident on the device."""

    def __init__(self, quick=False):
        import torch
        from . import inputs, segmented_sort
        d = 4 if quick else 1
        self.cases = {}
        # the ragged batch (u64 + payload, 10^7 geometric segments): a workload
        # of the global knobs and of the 64-bit lane-group mapping
        k, v, off = inputs.config4(nseg=10_000_000 // d, seed=44)
        to = torch.from_numpy(off).cuda()
        ragged = Case("ragged 10^7 u64+payload", lambda b: segmented_sort(b[0], to, b[1]),
                      [torch.from_numpy(k).cuda(), torch.from_numpy(v).cuda()],
                      24 * int(off[-1]) + 4 * (off.size - 1))
        del k, v
        for w in ("u32", "u64"):
            # (64-bit keys: the ragged batch too, whose RSS kernels finish with the family's networks)
            self.cases[(w, "family")] = ([_fixed_case(w, n, (1 << 22) // d, n) for n in (4, 8, 12, 16)]
                                         + [_csr_case(w, (1 << 18) // d, 17, 256, 5)]
                                         + ([ragged] if w == "u64" else []))
            self.cases[(w, "fixed_apt")] = [_fixed_case(w, n, (1 << 23) // d, n) for n in (2, 3, 4, 6, 8, 12, 16)]
            self.cases[(w, "fixed_half")] = None  # built one n at a time (fixed_half_case)
            # the mapping is tuned on the whole RSS range and on each group size's own range
            nr = (1 << 21) // d
            bounds = [_csr_case(w, (1 << 19) // d, 17, 256, 7), _csr_case(w, (1 << 18) // d, 17, 64, 8),
                      _csr_case(w, (1 << 18) // d, 65, 128, 10),
                      ragged if w == "u64" else
                      _csr_case(w, nr, 1, 256, 11, sizes=inputs.geometric_sizes(nr, 11), what="ragged, mean 24")]
            self.cases[(w, "rss_bound_tiny")] = bounds
            self.cases[(w, "rss_bound_small")] = bounds
            self.cases[(w, "rss_bound_mid")] = bounds
            self.cases[(w, "rss_k_small")] = [_csr_case(w, (1 << 18) // d, 17, 64, 64)]
            self.cases[(w, "rss_k_mid")] = [_csr_case(w, (1 << 18) // d, 65, 128, 128)]
            self.cases[(w, "rss_k_large")] = [_csr_case(w, (1 << 18) // d, 129, 256, 256)]
            self.cases[(w, "rss_oversample")] = [_csr_case(w, (1 << 19) // d, 17, 256, 9)]
            self.cases[(w, "rss_finish")] = self.cases[(w, "rss_oversample")]
        # global knobs: the ragged batch (u64 + payload) and the RSS-only batch (int32)
        k3, off3 = inputs.config3(nseg=(1 << 20) // d, dist="uniform", seed=7)
        to3 = torch.from_numpy(off3).cuda()
        rss = Case("RSS 2^20 int32", lambda b: segmented_sort(b[0], to3), [torch.from_numpy(k3).cuda()],
                   8 * int(off3[-1]) + 4 * (off3.size - 1))
        for g in GLOBAL:
            self.cases[("all", g)] = [ragged, rss]
        torch.cuda.synchronize()

    def all_cases(self):
        seen = {}
        for cs in self.cases.values():
            for c in cs or ():
                seen[id(c)] = c
        return list(seen.values())


def candidates(name):
    return {"family": [0, 1, 2], "fixed_apt": [1, 2, 4], "rss_bound_tiny": [16, 24, 32],
            "rss_bound_small": [16, 32, 48, 64],
            "rss_bound_mid": [64, 96, 128], "rss_k_small": [4, 8, 16], "rss_k_mid": [4, 8, 16, 32],
            "rss_k_large": [4, 8, 16, 32, 64], "rss_oversample": [1, 2, 3, 4], "rss_finish": [0, 1],
            "rss_rounds": [4, 8, 16, 32, 64],
            "persist_split": [0, 1], "net_mix": [0, 1], "interleave": [0, 1], "persist_occ": [0, 1, 2, 3]}[name]


def _tune_tile_threads(width, quick, reps, log):
    """Per n, the work-group size of the one-array-per-thread tile: 256 threads
    (no bit), 128 (bit n of fixed_half), 512 or 1024 over 256 arrays (bit n of
    fixed_wide or fixed_wider).  For each n the forms are compared on one fixed batch of that
    n (2^24 arrays and at least 512 MB, so that the Infinity Cache cannot hold
    it; a quarter in quick mode) with the other n as chosen so far: the
    networks are data-oblivious, so each sample times 8 back-to-back in-place
    calls, and `reps` samples of the forms alternate so that drift affects all
    alike.  Each form's output is checked against the library's default."""
    import torch
    from . import get_tuning, set_tuning
    d = 4 if quick else 1
    kb = 4 if width == "u32" else 8
    hn, wn, xn = f"{width}.fixed_half", f"{width}.fixed_wide", f"{width}.fixed_wider"
    half, wide, wider = get_tuning(hn), get_tuning(wn), get_tuning(xn)
    results, rejected = {}, []
    stream = torch.cuda.current_stream()

    def sample(case):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(8):
            case.call(case.bufs)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 8

    def apply(form, n):
        set_tuning(hn, (half & ~(1 << n)) | ((1 if form == 128 else 0) << n))
        set_tuning(wn, (wide & ~(1 << n)) | ((1 if form == 512 else 0) << n))
        set_tuning(xn, (wider & ~(1 << n)) | ((1 if form == 1024 else 0) << n))

    for n in range(2, 17):
        count = max(1 << 24, (1 << 29) // (n * kb)) // d
        case = _fixed_case(width, n, count, n)
        apply(256, n)
        case.record_reference()
        valid = []
        for form in (256, 128, 512, 1024):
            apply(form, n)
            case.restore()
            case.call(case.bufs)
            if case.output_matches():
                valid.append(form)
            else:
                rejected.append(f"n={n} threads={form}")
                log(f"  tile threads n={n} {form}: output differs from the reference -- rejected")
        samples = {form: [] for form in valid}
        for _ in range(reps):
            for form in valid:
                apply(form, n)
                samples[form].append(sample(case))
        times = {form: float(np.median(v)) for form, v in samples.items()}
        for form, ms in times.items():
            log(f"  {width} tile n={n} threads={form}: {ms:.4f} ms  {case.nbytes / (ms * 1e-3) / 1e9:.1f} GB/s")
        cur = 1024 if (wider >> n) & 1 else (512 if (wide >> n) & 1 else (128 if (half >> n) & 1 else 256))
        pick = min(times, key=times.get) if times else cur
        if cur in times and times[pick] > (1.0 - NOISE) * times[cur]:
            pick = cur
        half = (half & ~(1 << n)) | ((1 if pick == 128 else 0) << n)
        wide = (wide & ~(1 << n)) | ((1 if pick == 512 else 0) << n)
        wider = (wider & ~(1 << n)) | ((1 if pick == 1024 else 0) << n)
        apply(pick, n)
        results[f"n={n}"] = {"arrays": count, "ms_256": times.get(256), "ms_128": times.get(128),
                             "ms_512": times.get(512), "ms_1024": times.get(1024), "threads": pick}
        del case
        torch.cuda.empty_cache()
    set_tuning(hn, half)
    set_tuning(wn, wide)
    set_tuning(xn, wider)
    log(f"{hn} -> {half:#x}, {wn} -> {wide:#x}, {xn} -> {wider:#x}")
    return {hn: half, wn: wide, xn: wider}, {"workloads": [f"{width} fixed n=2..16"], "results": results,
                                             "rejected": rejected,
                                             "best": {"fixed_half": half, "fixed_wide": wide, "fixed_wider": wider}}


def tune(quick=False, reps=5, log=print):
    from . import SmallSortError, get_tuning, set_tuning
    w = Workloads(quick=quick)
    # reference outputs under the library's defaults (the tested configuration)
    for c in w.all_cases():
        c.record_reference()
    best, report = {}, {}
    order = [(wd, k) for wd in ("u32", "u64") for k in PER_WIDTH] + [("all", k) for k in GLOBAL]
    for width, knob in order:
        name = knob if width == "all" else f"{width}.{knob}"
        if knob == "fixed_half":  # with fixed_wide(r): one choice per n among four tile forms
            masks, report[f"{width}.tile_threads"] = _tune_tile_threads(width, quick, reps, log)
            best.update(masks)
            continue
        current = get_tuning(name)
        cases = w.cases[(width, knob)]
        results, rejected = {}, []
        for v in candidates(knob):
            try:
                set_tuning(name, v)
            except SmallSortError:
                continue  # not valid with the other current values (a bound pair)
            ms, ok = 0.0, True
            for c in cases:
                ms += c.time(reps)
                ok = ok and c.output_matches()
            if not ok:
                rejected.append(v)
                log(f"  {name}={v}: output differs from the reference -- rejected")
                continue
            nbytes = sum(c.nbytes for c in cases)
            results[v] = {"ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9}
            log(f"  {name}={v}: {ms:.4f} ms  {results[v]['GBps']:.1f} GB/s")
        choice = min(results, key=lambda v: results[v]["ms"]) if results else current
        if current in results and results[choice]["ms"] > (1.0 - NOISE) * results[current]["ms"]:
            choice = current
        set_tuning(name, choice)
        best[name] = choice
        report[name] = {"workloads": [c.name for c in cases], "results": {str(k): r for k, r in results.items()},
                        "rejected": rejected, "best": choice}
        log(f"{name} -> {choice}")
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
