"""Benchmark: batched small-array sorting on one MI355X.

Headline workload (the one the throughput target is stated for): 2^24 arrays
of n = 16 uint32 keys, uniform random, packed at stride 16, sorted in place by
one comparator network per array.  A step is one sort call over the whole
batch (one kernel launch) on its own fresh, unsorted copy of the input, which
is resident in HBM before the timed region starts.

Printed as one JSON line: keys/s, the roofline of the dominant kernel
(algorithmic HBM bytes per launch / its event-timed duration, against 8 TB/s),
HBM traffic per launch from the committed counter summary (only while the
kernel source is unchanged), and the CPU oracle timed on a bounded sample on
the host cores.  Unless --no-extras, the line also carries ``extras``: every
other workload --

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
                   choices=["all", "fixed16_u32", "config1", "config2", "rss", "rss_classes", "ragged", "serve"])
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extras", action="store_true", help="headline workload only")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    return p.parse_args()


# --- counters --------------------------------------------------------------------

# source files that define each profiled kernel's device code
KERNEL_SOURCES = {
    "fixed_tile_kernel<n=16,u32>": ("fixed.hip", "common.hpp", "networks_gen.hpp"),
}


def kernel_source_hash(kernel_key):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2002_05599_amd", "csrc")
    for f in KERNEL_SOURCES[kernel_key]:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, family):
    """HBM bytes per launch from profiles/traffic.json, if the counters were taken
    on the same kernel: unchanged sources and the same network family."""
    try:
        data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel_key) or ent.get("family") != family:
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
    kkey = "fixed_tile_kernel<n=16,u32>"
    family = ss.get_tuning("family")
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


def cpu_baseline_fixed(seconds, n=16):
    """The oracle (insertion sort at n <= 16) on a bounded sample, all host threads."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    count = 1 << 18
    src = np.random.default_rng(9).integers(0, 2**32, size=count * n, dtype=np.uint64).astype(np.uint32)
    oracle.sort_fixed(src[: n * 1024], n, 1024, n)
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.sort_fixed(src, n, count, n, threads=threads)  # sorts a fresh copy each pass
        done += count
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": done * n / el, "unit": "keys/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} arrays of {n} uint32 keys (uniform; one set of {count} arrays sorted "
                      f"from a fresh copy per pass), {threads} host threads, {el:.1f} s",
            "host": host_cpu()}


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


def bench_serve(args, pool=16, rhos=(0.5, 0.8), n_open=300):
    """Serving loop: saturated throughput, then Poisson arrivals at rho x saturation."""
    import torch
    from paper_2002_05599_amd import inputs
    from paper_2002_05599_amd.serve import GpuExecutor, SortServer, poisson_arrivals, run_open_loop

    jobs = [inputs.serving_request(i, seed=5) for i in range(pool)]
    mean_keys = float(np.mean([k.size for k, _ in jobs]))
    out = {"workload": f"serving, jobs of 1..100000 segments (sizes 2..256, uint32 uniform), "
                       f"pool of {pool} distinct jobs, Poisson arrivals, {n_open} jobs per load level",
           "mean_job_keys": mean_keys, "hbm_budget_bytes": 16 << 30}
    for where in ("device", "host"):
        if where == "device":
            pj = [(torch.from_numpy(k).cuda(), o) for k, o in jobs]
            torch.cuda.synchronize()
        else:
            pj = jobs
        ex = GpuExecutor(slots=3)

        def saturate():
            with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=8) as srv:
                hs = [srv.submit(*pj[i % pool]) for i in range(4 * pool)]
                for h in hs:
                    h.wait(600)
            return srv.stats()

        saturate()  # warm-up at full batch sizes: graphs, pinned buffers, workspaces, allocator pools
        sat = saturate()
        sat_rate = sat["jobs"] / sat["span_s"]
        # discarded open-loop pass: grows allocator pools and workspaces
        with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=8) as srv:
            run_open_loop(srv, pj, poisson_arrivals(n_open // 3, 0.5 * sat_rate, seed=4))
        res = {"saturated": {"jobs_per_s": sat_rate, "keys_per_s": sat["keys_per_s"]}}
        for rho in rhos:
            arr = poisson_arrivals(n_open, rho * sat_rate, seed=5)
            with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=8) as srv:
                run_open_loop(srv, pj, arr)
            st = srv.stats()
            res[f"rho_{rho}"] = {"offered_jobs_per_s": rho * sat_rate, "keys_per_s": st["keys_per_s"],
                                 "latency_ms": st["latency_ms"], "batches": st["batches"],
                                 "mean_jobs_per_batch": st["mean_jobs_per_batch"],
                                 "max_concurrent_batches": st["max_concurrent_batches"]}
        out[where] = res
        del pj, ex
        torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sorts shard into "
              "independent per-GPU batches with no communication, so a multi-GPU figure would be N "
              "copies of this one", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    w = args.workload
    if w in ("all", "fixed16_u32"):
        out = bench_fixed16(args)
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline_fixed(args.cpu_seconds)
        if w == "all" and not args.no_extras:
            ex = {}
            ex["config1"] = bench_config1(args)
            ex["config2"] = bench_config2(args)
            ex["config3_uniform"] = bench_rss(args, "uniform")
            ex["config3_zipf"] = bench_rss(args, "zipf")
            ex["config3_per_class"] = bench_rss_classes(args)
            ex["config4"] = bench_ragged(args)
            ex["config5"] = bench_serve(args)
            out["extras"] = ex
    elif w == "config1":
        out = bench_config1(args)
    elif w == "config2":
        out = bench_config2(args)
    elif w == "rss":
        out = {"rss_uniform": bench_rss(args, "uniform", steps=args.steps, warmup=args.warmup),
               "rss_zipf": bench_rss(args, "zipf", steps=args.steps, warmup=args.warmup)}
    elif w == "rss_classes":
        out = bench_rss_classes(args)
    elif w == "ragged":
        out = bench_ragged(args, steps=args.steps, warmup=args.warmup)
    else:
        out = bench_serve(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
