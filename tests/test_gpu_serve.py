"""Serving loop on the GPU: every job's result is the same alone and inside a mix."""
import numpy as np
import pytest

import oracle
from paper_2002_05599_amd import inputs
from paper_2002_05599_amd.serve import GpuExecutor, SortServer

pytestmark = pytest.mark.gpu


def small_jobs(n, seed, max_segments=3000):
    return [inputs.serving_request(i, seed=seed, max_segments=max_segments) for i in range(n)]


@pytest.fixture(scope="module")
def executor():
    import torch
    assert torch.cuda.is_available()
    return GpuExecutor(slots=3)


def run_alone(ex, jobs):
    out = []
    with SortServer(ex, max_batch_jobs=1) as srv:
        for k, o in jobs:
            out.append(srv.submit(k, o).wait(120))
    return out


def run_mix(ex, jobs, max_batch_jobs=6):
    with SortServer(ex, max_batch_jobs=max_batch_jobs) as srv:
        hs = [srv.submit(k, o) for k, o in jobs]
        out = [h.wait(120) for h in hs]
    return out, srv


def test_alone_equals_mix_host_jobs(executor):
    jobs = small_jobs(14, seed=5)
    alone = run_alone(executor, jobs)
    mix, srv = run_mix(executor, jobs)
    assert max(len(b) for b in srv.batches) > 1, "the mix must share batches"
    for (k, o), a, m in zip(jobs, alone, mix):
        want, _ = oracle.sort_segments(k, o)
        assert (a == want).all() and (m == want).all()


def test_alone_equals_mix_device_jobs(executor):
    import torch
    jobs = small_jobs(10, seed=6)
    dev = [(torch.from_numpy(k).cuda(), o) for k, o in jobs]
    torch.cuda.synchronize()
    alone = [r.cpu().numpy() for r in run_alone(executor, dev)]
    mix, srv = run_mix(executor, dev, max_batch_jobs=4)
    mix = [r.cpu().numpy() for r in mix]
    for (k, o), a, m in zip(jobs, alone, mix):
        want, _ = oracle.sort_segments(k, o)
        assert (a == want).all() and (m == want).all()
    # inputs are not modified (batches sort a gathered copy)
    for (k, _), (t, _) in zip(jobs, dev):
        assert (t.cpu().numpy() == k).all()


def test_batches_overlap_on_streams_and_budget_holds(executor):
    jobs = small_jobs(24, seed=7, max_segments=20000)
    budget = 6 * max(k.nbytes for k, _ in jobs)
    with SortServer(executor, hbm_budget=budget, max_batch_jobs=2) as srv:
        hs = [srv.submit(k, o) for k, o in jobs]
        for h in hs:
            h.wait(120)
    assert srv.max_concurrent_batches >= 2
    assert srv.max_inflight_bytes <= budget
    for (k, o), h in zip(jobs, hs):
        assert (h.result == oracle.sort_segments(k, o)[0]).all()
