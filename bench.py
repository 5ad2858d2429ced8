"""Benchmark: batched small-array sorting on one MI355X.

Headline workload (the one the throughput target is stated for): 2^24 arrays
of n = 16 uint32 keys, uniform random, packed at stride 16, sorted in place by
one comparator network per array.  A step is one sort call over the whole
batch (one kernel launch) on its own fresh, unsorted copy of the input, which
is resident in HBM before the timed region starts.

The LAST line on stdout is the compact headline JSON: keys/s, the roofline
of the dominant kernel (algorithmic HBM bytes per launch / its event-timed
duration, against 8 TB/s, beside the measured device-copy ceiling), HBM
traffic per launch from the committed counter summary (only while the
kernel source is unchanged), and the CPU oracle timed on a bounded sample on
the host cores.  Unless --no-extras, every other workload runs first and
prints one JSON line of its own (``{"extra": name, ...}``), and all of them
are also written to --extras-out:

  copy_ceiling  device-to-device copy of 1 GiB: runtime copy, streaming probe
  config1  100,000 arrays of 8 uint32 keys (launch-to-completion latency)
  config2  n = 2..16, 2^24 arrays, uint32 and int64, four distributions
  config3  Register Sample Sort, 2^20 CSR arrays of 17..256 int32 keys,
           uniform and Zipf(1.1); persistent graph vs per-class launches
  config4  10^7 ragged segments (geometric, mean 24), uint64 distinct keys +
           uint32 payload; persistent graph vs persistent vs per-class launches
  config5  the serving loop: saturated throughput, p50/p99 latency under
           Poisson arrivals at 0.5 and 0.8 of saturation

``--workload`` runs a single one of them (for profiling).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MALL_BYTES = 256 << 20  # Infinity Cache of one MI355X
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="all",
                   choices=["all", "fixed16_u32", "copy", "config1", "config2", "rss", "rss_classes", "ragged",
                            "serve", "is_vs_sn", "large"])
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extras", action="store_true", help="headline workload only")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--family", type=int, choices=(0, 1), default=None,
                   help="network family of the fixed-layout workloads (default: the tuned one)")
    p.add_argument("--extras-out", default=os.path.join(ROOT, "gpurun_out", "bench_extras.json"),
                   help="file for the extra workloads' results (also printed one per line)")
    return p.parse_args()


# --- counters --------------------------------------------------------------------

# source files that define each profiled kernel's device code
_FIXED_SOURCES = ("fixed.hip", "common.hpp", "keymap.hpp", "networks_gen.hpp")
KERNEL_SOURCES = {
    "fixed_tile_kernel<n=16,u32>": _FIXED_SOURCES,
    "fixed_half_tile_kernel<n=16,u32>": _FIXED_SOURCES,
    "fixed_wide_tile_kernel<n=16,u32>": _FIXED_SOURCES,
    "fixed_wider_tile_kernel<n=16,u32>": _FIXED_SOURCES,
}


def fixed16_kernel(ss):
    """The kernel that sorts 16-key uint32 arrays under the current tuning
    (the tile form chosen for n = 16)."""
    apt = ss.get_tuning("u32.fixed_apt")
    if apt >= 2:  # tiles of several arrays per thread (no counter record is kept for them)
        return f"fixed_tile_kernel<n=16,u32,{apt} arrays per thread>"
    if (ss.get_tuning("u32.fixed_wider") >> 16) & 1:
        return "fixed_wider_tile_kernel<n=16,u32>"
    if (ss.get_tuning("u32.fixed_wide") >> 16) & 1:
        return "fixed_wide_tile_kernel<n=16,u32>"
    if (ss.get_tuning("u32.fixed_half") >> 16) & 1:
        return "fixed_half_tile_kernel<n=16,u32>"
    return "fixed_tile_kernel<n=16,u32>"


def kernel_source_hash(kernel_key):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2002_05599_amd", "csrc")
    for f in KERNEL_SOURCES[kernel_key]:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, family):
    """HBM bytes per launch from profiles/traffic.json, if the counters were taken
    on the same kernel: unchanged sources and the same network family (one
    record per family)."""
    try:
        data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    except (OSError, ValueError):
        return None
    if kernel_key not in KERNEL_SOURCES:
        return None
    ent = data.get(kernel_key, {}).get(f"family {family}")
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel_key):
        return None
    return ent.get("bytes_per_launch")


# --- timing helpers ----------------------------------------------------------------

class StepBuffers:
    """``count`` device copies of a pristine input, restored (untimed) on demand."""

    def __init__(self, pristine, count):
        self.pristine = pristine
        self.bufs = [tuple(t.clone() for t in pristine) for _ in range(count)]

    def restore(self):
        import torch
        for b in self.bufs:
            for dst, src in zip(b, self.pristine):
                dst.copy_(src)
        torch.cuda.synchronize()


def time_steps(step, bufs, steps, warmup):
    """Warm up, restore every copy, then time exactly ``steps`` steps (one fresh
    copy each) between two synchronisations, with events on the stream."""
    import torch
    for i in range(warmup):
        step(bufs.bufs[i % len(bufs.bufs)])
    bufs.restore()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(steps):
        step(bufs.bufs[i])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall


def time_inplace(step, steps, warmup):
    """Events around ``steps`` back-to-back calls on one buffer (data-oblivious sorts)."""
    import torch
    for _ in range(warmup):
        step()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def rate(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}


# --- workloads ---------------------------------------------------------------------

def bench_fixed16(args):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs

    n, count_log2 = 16, 24
    count = 1 << count_log2
    keys = torch.from_numpy(inputs.fixed_keys(np.uint32, n, count, "uniform", seed=2)).cuda()
    bufs = StepBuffers((keys,), args.steps)
    ms, wall = time_steps(lambda b: ss.sort_small(b[0], n), bufs, args.steps, args.warmup)
    nkeys = count * n
    algo_bytes = 2 * nkeys * 4
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    kkey = fixed16_kernel(ss)
    family = ss.get_tuning("u32.family")
    del bufs, keys
    torch.cuda.empty_cache()
    return {
        "metric": "keys/s", "value": nkeys / (ms * 1e-3), "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched network sort, 2^{count_log2} arrays x n={n} uint32, uniform, "
                               f"stride {n}", "n": n, "count": count, "key": "uint32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(kkey, family),
                     "kernel": kkey, "network_family": family, "algorithmic_bytes_per_launch": algo_bytes},
    }


def cpu_share():
    """Host threads this process may use: its CPU affinity, capped at the CPU
    share of a one-GPU job on the MI355X hosts (16 threads)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, 16))


def cpu_baseline_fixed(seconds, n=16):
    """The oracle (insertion sort at n <= 16) timed on a bounded sample of the
    headline workload: built with gcc -O3 -march=native on this host (the
    paper's compiler settings, Section 4.1), run (a) on one thread pinned to
    one core, like the paper's taskset runs, and (b) on every thread of this
    process's CPU share.  Each pass sorts a fresh copy of the sample in place;
    the copy is restored outside the timed region.  Median of the passes."""
    import tempfile
    import oracle
    from oracle import build as oracle_build
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    lib = oracle.load(oracle_build.build_native(os.path.join(tmp, "liboracle_native.so")))
    count = 1 << 18  # 4 M keys, 16 MiB: far above the host's last-level cache per core
    src = np.random.default_rng(9).integers(0, 2**32, size=count * n, dtype=np.uint64).astype(np.uint32)
    work = src.copy()

    def run(threads, budget):
        oracle.sort_fixed_inplace(work, n, count, n, lib=lib, threads=threads)  # warm-up
        times = []
        t_end = time.perf_counter() + budget
        while len(times) < 3 or (time.perf_counter() < t_end and len(times) < 200):
            np.copyto(work, src)
            t0 = time.perf_counter()
            oracle.sort_fixed_inplace(work, n, count, n, lib=lib, threads=threads)
            times.append(time.perf_counter() - t0)
        return count * n / float(np.median(times)), len(times)

    cores = cpu_share()
    single_core = None
    old_aff = None
    try:
        old_aff = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old_aff)})
        single_core = min(old_aff)
    except (AttributeError, OSError):
        pass
    try:
        one, n_one = run(1, seconds * 0.6)
    finally:
        if old_aff is not None:
            os.sched_setaffinity(0, old_aff)
    many, n_many = run(cores, seconds * 0.4)
    return {"value": many, "unit": "keys/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} arrays x {n} uint32 keys (16 MiB, uniform), in place, median of {n_many} "
                      f"passes on {cores} threads; single thread pinned to core {single_core}: "
                      f"{one:.4g} keys/s ({n_one} passes); gcc -O3 -march=native",
            "single_thread_value": one, "host": host_cpu()}


def host_cpu():
    """Model name and logical CPU count of the host that ran the oracle."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def bench_copy_ceiling(args, nbytes=1 << 30, steps=20, warmup=3):
    """Device-to-device copy of 1 GiB (2 GiB moved): the runtime's copy and the
    library's streaming copy probe -- the practical ceiling of a kernel that
    reads and writes every byte once."""
    import torch
    import paper_2002_05599_amd as ss
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").random_()
    dst = torch.empty_like(src)
    out = {}
    for name, fn in (("runtime_copy", lambda: dst.copy_(src)), ("stream_copy", lambda: ss.stream_copy(dst, src))):
        ms = time_inplace(fn, steps, warmup)
        out[name] = {"ms": ms, **rate(2 * nbytes, ms)}
    assert torch.equal(dst, src)
    del src, dst
    torch.cuda.empty_cache()
    return {"workload": "device-to-device copy of 1 GiB (2 GiB moved)", **out}


def bench_config1(args):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs
    a = torch.from_numpy(inputs.config1()).cuda()
    ms = time_inplace(lambda: ss.sort_small(a, 8), 50, 10)
    lat = []  # launch-to-completion latency of one call, host clock
    for _ in range(50):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ss.sort_small(a, 8)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    return {"workload": "100,000 arrays x n=8 uint32, uniform (3.2 MB, cache resident)",
            "kernel_ms": ms, "keys_per_s": 8e5 / (ms * 1e-3),
            "call_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "note": "fits in L2/MALL: latency-bound, % of HBM not meaningful"}


def device_fixed_keys(torch, dtype, n, count, dist, gen):
    """Device-side random input of the given distribution (timing only)."""
    shape = (count, n)
    if dist == "uniform":
        if dtype == "u32":
            return torch.randint(-2**31, 2**31 - 1, shape, dtype=torch.int32, device="cuda",
                                 generator=gen).view(torch.uint32)
        return torch.randint(-2**63, 2**63 - 1, shape, dtype=torch.int64, device="cuda", generator=gen)
    if dist == "few":
        x = torch.randint(0, 4, shape, dtype=torch.int32, device="cuda", generator=gen)
        return x.view(torch.uint32) if dtype == "u32" else x.to(torch.int64)
    # sorted / reverse: base + j*2^20 + r_j with r_j < 2^20 is increasing in j
    x = torch.randint(0, 1 << 20, shape, dtype=torch.int64, device="cuda", generator=gen)
    x += torch.arange(n, dtype=torch.int64, device="cuda").view(1, n) << 20
    x += torch.randint(0, 1 << 20, (count, 1), dtype=torch.int64, device="cuda", generator=gen)
    if dist == "reverse":
        x = torch.flip(x, dims=[1])
    x = x.contiguous()
    return x.to(torch.int32).view(torch.uint32) if dtype == "u32" else x


def bench_config2(args):
    """Networks for every n = 2..16, 2^24 arrays, u32 and i64, four distributions."""
    import torch
    import paper_2002_05599_amd as ss
    count = 1 << 24
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    out = {}
    for dtype, kb in (("u32", 4), ("i64", 8)):
        for n in range(2, 17):
            row = {}
            for dist in ("uniform", "few", "sorted", "reverse"):
                a = device_fixed_keys(torch, dtype, n, count, dist, gen).reshape(-1)
                # footprints that fit the 256 MB MALL rotate over 4 buffers (1 GiB), so
                # every call streams from HBM
                bufs = [a] if count * n * kb > MALL_BYTES else [a] + [a.clone() for _ in range(3)]
                calls = [0]

                def step():
                    ss.sort_small(bufs[calls[0] % len(bufs)], n)
                    calls[0] += 1

                ms = time_inplace(step, 8, 4)
                row[dist] = {"ms": ms, "keys_per_s": count * n / (ms * 1e-3), **rate(2 * count * n * kb, ms),
                             "buffers": len(bufs)}
                del a, bufs
            out[f"{dtype}_n{n}"] = row
    torch.cuda.empty_cache()
    return {"workload": "2^24 arrays per n, stride n; time per call (the networks are data-oblivious, "
                        "so repeated in-place calls do identical work); inputs of at most 256 MB rotate "
                        "over 4 buffers", "results": out}


def bench_network_vs_insertion(args):
    """The paper's central comparison (Sections 4.2-4.3, ArrayInRow): for each
    n = 2..16, the fastest network family against insertion sort ("IS Def",
    family 2), 2^24 arrays per n, uint32 and int64, uniform and already-sorted
    rows (insertion sort is adaptive, the networks are not).  Above 16 keys:
    Register Sample Sort with network and with insertion-sort base cases
    (Section 4.5) and the IS+SN hybrid (Section 4.6: insertion sort for every
    array above 16 keys) on the 2^20-array RSS batch."""
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs
    count = 1 << 24
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    rows = {}
    with ss.tuned(family=0):
        for dtype, kb in (("u32", 4), ("i64", 8)):
            for n in range(2, 17):
                row = {}
                for dist in ("uniform", "sorted"):
                    src = device_fixed_keys(torch, dtype, n, count, dist, gen).reshape(-1)
                    buf = src.clone()
                    ms = {}
                    for fam in (0, 1, 2):
                        ss.set_tuning("family", fam)
                        # insertion sort is adaptive: every call gets a fresh copy of the
                        # input (for small n the copy leaves it in the Infinity Cache;
                        # every variant sees the same, so the ratio stands)
                        ms[fam] = time_restored(lambda: ss.sort_small(buf, n), lambda: buf.copy_(src), 5)
                    best_net = min(ms[0], ms[1])
                    row[dist] = {"best_network_ms": best_net, "best_family": 0 if ms[0] <= ms[1] else 1,
                                 "insertion_ms": ms[2], "network_speedup": ms[2] / best_net}
                    del src, buf
                rows[f"{dtype}_n{n}"] = row

    torch.cuda.empty_cache()
    # 17..256 keys: RSS (network base case), RSS with insertion-sort base case, IS+SN
    keys, off = inputs.config3(nseg=1 << 20, dist="uniform")
    tk = torch.from_numpy(keys).cuda()
    to = torch.from_numpy(off).cuda()
    bufs = StepBuffers((tk,), 3)
    large = {}
    for name, knobs in (("rss_network_base", {}), ("rss_insertion_base", {"family": 2}),
                        ("is_sn_hybrid", {"large_sort": 1})):
        with ss.tuned(**knobs):
            ms, _ = time_steps(lambda b: ss.segmented_sort(b[0], to), bufs, 3, 1)
        large[name] = {"ms": ms}
    for name in large:
        large[name]["speedup_of_rss_network_base"] = large[name]["ms"] / large["rss_network_base"]["ms"]
    assert ss.device_status() == 0
    del bufs, tk, to
    torch.cuda.empty_cache()
    return {"workload": "networks vs insertion sort: 2^24 arrays per n = 2..16 (u32, i64; uniform and sorted "
                        "rows); above 16 keys the 2^20-array RSS batch (int32 uniform, graph form)",
            "per_n": rows, "above_16": large}


def time_restored(step, restore, calls, warmup=2):
    """Median over ``calls`` calls of the event-timed duration of one call,
    each on a freshly restored input (``restore`` runs untimed before it)."""
    import torch
    for _ in range(warmup):
        restore()
        step()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(calls):
        restore()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        step()
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    return float(np.median(times))


def bench_large_and_device_sort(args):
    """Above 256 keys: arrays of 512..4096 keys in the fixed layout (one
    work-group per array, runs merged in LDS), and the device-wide sort with the
    small sorters as base case, on 2^28 uint32 keys and on 2^26 uint64 keys with
    uint64 references (the paper's items)."""
    import torch
    import paper_2002_05599_amd as ss
    gen = torch.Generator(device="cuda")
    gen.manual_seed(21)
    large = {}
    for n in (512, 1024, 2048, 4096):
        count = (1 << 26) // n
        src = torch.randint(-2**31, 2**31 - 1, (count * n,), dtype=torch.int32, device="cuda",
                            generator=gen).view(torch.uint32)
        buf = src.clone()
        ms = time_restored(lambda: ss.sort_small(buf, n), lambda: buf.copy_(src), 5)
        large[f"u32_n{n}"] = {"count": count, "ms": ms, "keys_per_s": count * n / (ms * 1e-3),
                              **rate(8 * count * n, ms)}
        del src, buf
    dev = {}
    for name, n, kdt, vdt in (("u32_2p28", 1 << 28, torch.int32, None),
                              ("u64_u64ref_2p26", 1 << 26, torch.int64, torch.int64)):
        lo, hi = (-2**31, 2**31 - 1) if kdt == torch.int32 else (-2**63, 2**63 - 1)
        src = torch.randint(lo, hi, (n,), dtype=kdt, device="cuda", generator=gen)
        src = src.view(torch.uint32 if kdt == torch.int32 else torch.uint64)
        vsrc = (torch.arange(n, dtype=torch.int64, device="cuda").view(torch.uint64) if vdt is not None else None)
        kb = src.element_size() + (8 if vdt is not None else 0)
        k = src.clone()
        v = vsrc.clone() if vsrc is not None else None
        ws = torch.empty(ss.sort_workspace_bytes("uint32" if kdt == torch.int32 else "uint64", n,
                                                 8 if vdt is not None else 0), dtype=torch.uint8, device="cuda")

        def restore():
            k.copy_(src)
            if v is not None:
                v.copy_(vsrc)

        ms = time_restored(lambda: ss.sort(k, v, workspace=ws), restore, 3, warmup=1)
        dev[name] = {"n": n, "ms": ms, "keys_per_s": n / (ms * 1e-3), **rate(2 * kb * n, ms)}
        del src, vsrc, k, v, ws
    torch.cuda.empty_cache()
    assert ss.device_status() == 0
    return {"workload": "fixed-layout arrays of 512..4096 uint32 keys (2^26 keys per size); device-wide sort "
                        "of 2^28 uint32 keys and of 2^26 uint64 keys + uint64 references, uniform random "
                        "(one call includes its stream synchronisations)", "large_arrays": large,
            "device_sort": dev}


def seg_bytes(total, nseg, key_bytes, has_vals):
    return 2 * total * (key_bytes + (4 if has_vals else 0)) + 4 * (nseg + 1)


def bench_rss(args, dist="uniform", nseg=1 << 20, steps=10, warmup=2):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs
    keys, off = inputs.config3(nseg=nseg, dist=dist)
    total = int(off[-1])
    tk = torch.from_numpy(keys).cuda()
    to = torch.from_numpy(off).cuda()
    bufs = StepBuffers((tk,), steps)
    res = {}
    for name, mode in (("graph", ss.MODE_AUTO), ("plain", ss.MODE_PLAIN)):
        ms, _ = time_steps(lambda b: ss.segmented_sort(b[0], to, mode=mode), bufs, steps, warmup)
        res[name] = {"ms": ms, "keys_per_s": total / (ms * 1e-3), **rate(seg_bytes(total, nseg, 4, False), ms)}
    assert ss.device_status() == 0
    del bufs
    torch.cuda.empty_cache()
    return {"workload": f"RSS, {nseg} CSR arrays, n uniform in [17,256], int32 {dist}", "keys": total,
            "nseg": nseg, **res}


def bench_rss_classes(args, nseg=1 << 20, steps=5, warmup=2):
    """2^20 CSR arrays per size class (17..32, 33..64, 65..128, 129..256), int32 uniform."""
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs
    out = {}
    for lo, hi in ((17, 32), (33, 64), (65, 128), (129, 256)):
        off = inputs.offsets_from_sizes(inputs.csr_sizes(nseg, lo, hi, seed=hi))
        total = int(off[-1])
        tk = torch.from_numpy(inputs.random_keys(np.int32, total, seed=lo)).cuda()
        to = torch.from_numpy(off).cuda()
        bufs = StepBuffers((tk,), steps)
        row = {}
        for name, mode in (("graph", ss.MODE_AUTO), ("plain", ss.MODE_PLAIN)):
            ms, _ = time_steps(lambda b: ss.segmented_sort(b[0], to, mode=mode), bufs, steps, warmup)
            row[name] = {"ms": ms, "keys_per_s": total / (ms * 1e-3), **rate(seg_bytes(total, nseg, 4, False), ms)}
        out[f"{lo}..{hi}"] = {"keys": total, **row}
        del bufs, tk, to
        torch.cuda.empty_cache()
    assert ss.device_status() == 0
    return {"workload": f"RSS per size class, {nseg} CSR arrays each, n uniform in the class, int32 uniform",
            "classes": out}


def bench_ragged(args, nseg=10_000_000, steps=10, warmup=2):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs
    keys, vals, off = inputs.config4(nseg=nseg)
    total = int(off[-1])
    tk = torch.from_numpy(keys).cuda()
    tv = torch.from_numpy(vals).cuda()
    to = torch.from_numpy(off).cuda()
    bufs = StepBuffers((tk, tv), steps)
    res = {}
    for name, mode in (("graph", ss.MODE_AUTO), ("persistent", ss.MODE_PERSISTENT), ("plain", ss.MODE_PLAIN)):
        ms, _ = time_steps(lambda b: ss.segmented_sort(b[0], to, b[1], mode=mode), bufs, steps, warmup)
        res[name] = {"ms": ms, "keys_per_s": total / (ms * 1e-3), **rate(seg_bytes(total, nseg, 8, True), ms)}
    assert ss.device_status() == 0
    res["graph_speedup_vs_plain"] = res["plain"]["ms"] / res["graph"]["ms"]
    del bufs
    torch.cuda.empty_cache()
    return {"workload": f"ragged, {nseg} segments, geometric sizes (mean 24, 1..256), uint64 distinct keys "
                        f"+ uint32 payload; every form includes its size-class binning", "keys": total,
            "nseg": nseg, **res}


def bench_serve(args, pool=16, rhos=(0.5, 0.8), n_open=300, batch_jobs=8, window_s=2e-4):
    """Serving loop.  For device-resident jobs, saturation is the device's own
    rate on the job pool (batches of ``batch_jobs`` jobs back to back on one
    stream, timed with HIP events, so it does not follow the host's load);
    for host jobs, whose bound is the host's staging copies, it is the
    server's closed-loop rate.  Poisson arrivals are
    then offered at rho x saturation and each job's latency is measured from
    its scheduled arrival (a client that falls behind its schedule shows the
    delay instead of hiding it).  Device-resident jobs (keys already in HBM)
    and host jobs (PCIe both ways) are run separately."""
    import torch
    from paper_2002_05599_amd import inputs
    from paper_2002_05599_amd.serve import GpuExecutor, SortServer, poisson_arrivals, run_open_loop

    jobs = [inputs.serving_request(i, seed=5) for i in range(pool)]
    mean_keys = float(np.mean([k.size for k, _ in jobs]))
    out = {"workload": f"serving, jobs of 1..100000 segments (sizes 2..256, uint32 uniform), "
                       f"pool of {pool} distinct jobs, Poisson arrivals, {n_open} jobs per load level, "
                       f"batching window {window_s * 1e6:.0f} us, at most {batch_jobs} jobs per batch",
           "mean_job_keys": mean_keys, "hbm_budget_bytes": 16 << 30}
    for where in ("device", "host"):
        if where == "device":
            pj = [(torch.from_numpy(k).cuda(), o) for k, o in jobs]
            torch.cuda.synchronize()
        else:
            pj = jobs
        ex = GpuExecutor(slots=3)
        ex.device_rate(pj, batch_jobs, reps=1)  # warm-up: workspaces, graphs, allocator pools
        if where == "device":
            sat_rate = ex.device_rate(pj * 4, batch_jobs, reps=3)
            sat_kind = "saturated_device"
        else:
            # host jobs are bound by the host's staging copies into pinned memory
            # and back, not by the device: their saturation is the server's own
            # closed-loop rate (all jobs queued at once)
            def closed_loop():
                with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=batch_jobs) as srv:
                    for h in [srv.submit(*pj[i % pool]) for i in range(4 * pool)]:
                        h.wait(600)
                return srv.stats()
            closed_loop()
            st = closed_loop()
            sat_rate = st["jobs"] / st["span_s"]
            sat_kind = "saturated_server_closed_loop"
        # discarded open-loop pass at the lower load: pinned buffers, per-stream workspaces
        with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=batch_jobs, batch_window_s=window_s) as srv:
            run_open_loop(srv, pj, poisson_arrivals(n_open // 3, rhos[0] * sat_rate, seed=4))
        res = {sat_kind: {"jobs_per_s": sat_rate, "keys_per_s": sat_rate * mean_keys}}
        for rho in rhos:
            arr = poisson_arrivals(n_open, rho * sat_rate, seed=5)
            with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=batch_jobs, batch_window_s=window_s) as srv:
                run_open_loop(srv, pj, arr)
            st = srv.stats()
            res[f"rho_{rho}"] = {"offered_jobs_per_s": rho * sat_rate, "keys_per_s": st["keys_per_s"],
                                 "latency_ms_from_scheduled_arrival": st["latency_ms"], "batches": st["batches"],
                                 "mean_jobs_per_batch": st["mean_jobs_per_batch"],
                                 "max_concurrent_batches": st["max_concurrent_batches"],
                                 "max_inflight_bytes": st["max_inflight_bytes"]}
        out[where] = res
        del pj, ex
        torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def compact(x, digits=4):
    """Round floats so the extras lines stay short."""
    if isinstance(x, float):
        return float(f"{x:.{digits}g}")
    if isinstance(x, dict):
        return {k: compact(v, digits) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [compact(v, digits) for v in x]
    return x


EXTRAS = [
    ("config1", bench_config1),
    ("config2", bench_config2),
    ("network_vs_insertion", bench_network_vs_insertion),
    ("large_and_device_sort", bench_large_and_device_sort),
    ("config3_uniform", lambda a: bench_rss(a, "uniform")),
    ("config3_zipf", lambda a: bench_rss(a, "zipf")),
    ("config3_per_class", bench_rss_classes),
    ("config4", bench_ragged),
    ("config5", bench_serve),
]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sorts shard into "
              "independent per-GPU batches with no communication, so a multi-GPU figure would be N "
              "copies of this one", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.family is not None:
        import paper_2002_05599_amd as ss
        ss.set_tuning("family", args.family)
    w = args.workload
    if w in ("all", "fixed16_u32"):
        ceiling = bench_copy_ceiling(args)
        out = bench_fixed16(args)
        out["roofline"]["copy_ceiling_GBps"] = {k: round(ceiling[k]["GBps"], 1)
                                                for k in ("runtime_copy", "stream_copy")}
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline_fixed(args.cpu_seconds)
        if w == "all" and not args.no_extras:
            extras = {"copy_ceiling": ceiling}
            print(json.dumps({"extra": "copy_ceiling", **compact(ceiling)}), flush=True)
            for name, fn in EXTRAS:
                res = compact(fn(args))
                extras[name] = res
                print(json.dumps({"extra": name, **res}), flush=True)
            if args.extras_out:
                os.makedirs(os.path.dirname(os.path.abspath(args.extras_out)), exist_ok=True)
                with open(args.extras_out, "w") as f:
                    json.dump(extras, f, indent=1)
                out["extras_file"] = args.extras_out
    elif w == "copy":
        out = bench_copy_ceiling(args)
    elif w == "config1":
        out = bench_config1(args)
    elif w == "config2":
        out = bench_config2(args)
    elif w == "rss":
        out = {"rss_uniform": bench_rss(args, "uniform", steps=args.steps, warmup=args.warmup),
               "rss_zipf": bench_rss(args, "zipf", steps=args.steps, warmup=args.warmup)}
    elif w == "rss_classes":
        out = bench_rss_classes(args)
    elif w == "large":
        out = bench_large_and_device_sort(args)
    elif w == "is_vs_sn":
        out = bench_network_vs_insertion(args)
    elif w == "ragged":
        out = bench_ragged(args, steps=args.steps, warmup=args.warmup)
    else:
        out = bench_serve(args)
    # the headline is the last line on stdout, compact
    print(json.dumps(compact(out, 6), separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
