"""Benchmark: batched small-array sorting on one MI355X.

Default workload (the one the throughput target is stated for): 2^24 arrays
of n = 16 uint32 keys, uniform random, packed at stride 16, sorted in place by
one comparator network per array.  A step is one sort call over the whole
batch (one kernel launch).  The network is data-oblivious -- every step runs
the same instructions and moves the same bytes whatever the data -- so the
steps after the first re-sort the same, now sorted, buffer at identical cost.

Prints one JSON line: keys/s, the roofline of the dominant kernel (algorithmic
HBM bytes per launch / its event-timed duration vs 8 TB/s), and the CPU oracle
timed on a bounded sample on the host cores.

Other workloads (``--workload``): rss (2^20 CSR arrays of 17..256 int32 keys),
ragged (10^7 geometric segments, uint64 keys + uint32 payload; persistent
graph launch and the plain per-class baseline), serve (the serving loop).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="fixed16_u32",
                   choices=["fixed16_u32", "rss", "ragged", "serve"])
    p.add_argument("--n", type=int, default=16)
    p.add_argument("--count-log2", type=int, default=24)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2002_05599_amd", "csrc"))):
        if f.endswith((".hip", ".hpp")):
            h.update(open(os.path.join(ROOT, "paper_2002_05599_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key):
    """HBM bytes per launch from the committed counter summary, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline_fixed(n, dtype, seconds):
    """Oracle (insertion sort, n <= 16) on a bounded sample, all host threads."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    count = 1 << 18
    a = np.ascontiguousarray(np.random.default_rng(9).integers(0, 2**32, size=count * n, dtype=np.uint64)
                             .astype(dtype))
    oracle.sort_fixed(a[: n * 1024], n, 1024, n)  # load + warm
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.sort_fixed(a, n, count, n, threads=threads)
        done += count
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": done * n / el, "unit": "keys/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} arrays of {n} {np.dtype(dtype).name} keys (uniform), "
                      f"{threads} host threads, {el:.1f} s"}


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
    """Run warmup steps, restore every copy, then time exactly ``steps`` steps
    (one fresh copy each) between two synchronisations and two events."""
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


def bench_fixed(args):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs

    n = args.n
    count = 1 << args.count_log2
    keys = torch.from_numpy(inputs.fixed_keys(np.uint32, n, count, "uniform", seed=2)).cuda()
    bufs = StepBuffers((keys,), args.steps)
    ms, wall = time_steps(lambda b: ss.sort_small(b[0], n), bufs, args.steps, args.warmup)
    nkeys = count * n
    algo_bytes = 2 * nkeys * 4
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    kkey = f"fixed_tile_kernel<n={n},u32>"
    out = {
        "metric": "keys/s", "value": nkeys / (ms * 1e-3), "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "wall_s_timed": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched network sort, 2^{args.count_log2} arrays x n={n} uint32, "
                               f"uniform, stride {n}", "n": n, "count": count, "key": "uint32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(kkey),
                     "kernel": kkey, "algorithmic_bytes_per_launch": algo_bytes},
    }
    return out, (n, np.uint32)


def seg_bytes(total, nseg, key_bytes, has_vals):
    return 2 * total * (key_bytes + (4 if has_vals else 0)) + 4 * (nseg + 1)


def bench_rss(args, dist="uniform", nseg=1 << 20):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs

    keys, off = inputs.config3(nseg=nseg, dist=dist)
    total = int(off[-1])
    tk = torch.from_numpy(keys).cuda()
    to = torch.from_numpy(off).cuda()
    bufs = StepBuffers((tk,), args.steps)
    res = {}
    for name, mode in (("graph", ss.MODE_AUTO), ("plain", ss.MODE_PLAIN)):
        ms, wall = time_steps(lambda b: ss.segmented_sort(b[0], to, mode=mode), bufs, args.steps, args.warmup)
        gbs = seg_bytes(total, nseg, 4, False) / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "keys_per_s": total / (ms * 1e-3), "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    assert ss.device_status() == 0
    return {"workload": f"RSS, {nseg} CSR arrays, n uniform in [17,256], int32 {dist}", "keys": total,
            "nseg": nseg, **res}


def bench_ragged(args, nseg=10_000_000):
    import torch
    import paper_2002_05599_amd as ss
    from paper_2002_05599_amd import inputs

    keys, vals, off = inputs.config4(nseg=nseg)
    total = int(off[-1])
    tk = torch.from_numpy(keys).cuda()
    tv = torch.from_numpy(vals).cuda()
    to = torch.from_numpy(off).cuda()
    bufs = StepBuffers((tk, tv), args.steps)
    res = {}
    for name, mode in (("graph", ss.MODE_AUTO), ("persistent", ss.MODE_PERSISTENT), ("plain", ss.MODE_PLAIN)):
        ms, wall = time_steps(lambda b: ss.segmented_sort(b[0], to, b[1], mode=mode), bufs, args.steps,
                              args.warmup)
        gbs = seg_bytes(total, nseg, 8, True) / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "keys_per_s": total / (ms * 1e-3), "GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    assert ss.device_status() == 0
    res["graph_speedup_vs_plain"] = res["plain"]["ms"] / res["graph"]["ms"]
    return {"workload": f"ragged, {nseg} segments, geometric sizes (mean 24, 1..256), uint64 distinct keys "
                        f"+ uint32 payload", "keys": total, "nseg": nseg, **res}


def bench_serve(args, pool=16, rhos=(0.5, 0.8), n_open=300):
    """Serving loop: saturated throughput, then Poisson arrivals at rho x saturation."""
    import torch
    from paper_2002_05599_amd import inputs
    from paper_2002_05599_amd.serve import GpuExecutor, SortServer, poisson_arrivals, run_open_loop

    jobs = [inputs.serving_request(i, seed=5) for i in range(pool)]
    mean_keys = float(np.mean([k.size for k, _ in jobs]))
    out = {"workload": f"serving, jobs of 1..100000 segments (sizes 2..256, uint32 uniform), "
                       f"pool of {pool} distinct jobs, Poisson arrivals",
           "mean_job_keys": mean_keys, "hbm_budget_bytes": 16 << 30}
    for where in ("device", "host"):
        if where == "device":
            pj = [(torch.from_numpy(k).cuda(), o) for k, o in jobs]
            torch.cuda.synchronize()
        else:
            pj = jobs
        ex = GpuExecutor(slots=3)
        with SortServer(ex, hbm_budget=16 << 30) as srv:  # warm-up: graphs, pinned buffers
            for i in range(3):
                srv.submit(*pj[i]).wait(600)
        with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=8) as srv:
            hs = [srv.submit(*pj[i % pool]) for i in range(4 * pool)]
            for h in hs:
                h.wait(600)
        sat = srv.stats()
        sat_rate = sat["jobs"] / sat["span_s"]
        # discarded open-loop pass: grows allocator pools and workspaces
        with SortServer(ex, hbm_budget=16 << 30, max_batch_jobs=8) as srv:
            run_open_loop(srv, pj, poisson_arrivals(n_open // 3, 0.5 * sat_rate, seed=4))
        res = {"saturated": {"jobs_per_s": sat_rate, "keys_per_s": sat["keys_per_s"],
                             "latency_ms": sat["latency_ms"]}}
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
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the sorts shard into independent per-GPU batches with no communication", file=sys.stderr)
        sys.exit(2)
    if args.workload == "fixed16_u32":
        out, (n, dt) = bench_fixed(args)
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline_fixed(n, dt, args.cpu_seconds)
    elif args.workload == "rss":
        out = {"rss_uniform": bench_rss(args, "uniform"), "rss_zipf": bench_rss(args, "zipf")}
    elif args.workload == "ragged":
        out = bench_ragged(args)
    else:
        out = bench_serve(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
