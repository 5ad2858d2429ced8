"""Serving loop scheduling, admission and accounting on the host (no GPU).

A host-only executor (the CPU oracle behind the executor interface, with an
artificial service time) stands in for the GPU.
"""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2002_05599_amd import inputs
from paper_2002_05599_amd.serve import AdmissionError, SortServer, build_batch, device_bytes


class FakeExecutor:
    def __init__(self, slots=2, service_s=0.005, fail_on=None):
        self.busy = [False] * slots
        self.service_s = service_s
        self.fail_on = fail_on
        self.inflight = {}
        self.launches = 0
        self.concurrent_max = 0
        self.key_bytes = 4

    def free_slot(self):
        for i, b in enumerate(self.busy):
            if not b:
                return i
        return None

    def launch(self, slot, jobs):
        self.launches += 1
        if self.fail_on is not None and self.launches == self.fail_on:
            raise RuntimeError("injected executor failure")
        self.busy[slot] = True
        keys, offsets, starts = build_batch(jobs)
        out, _ = oracle.sort_segments(keys, offsets)
        parts = [out[starts[i]:starts[i + 1]] for i in range(len(jobs))]
        self.inflight[slot] = (time.monotonic() + self.service_s, parts)
        self.concurrent_max = max(self.concurrent_max, sum(self.busy))

    def done(self, slot):
        return time.monotonic() >= self.inflight[slot][0]

    def result(self, slot):
        _, out = self.inflight.pop(slot)
        self.busy[slot] = False
        return out


def make_job(rng, nseg_max=200):
    nseg = int(rng.integers(1, nseg_max))
    sizes = rng.integers(2, 257, size=nseg)
    off = inputs.offsets_from_sizes(sizes)
    keys = rng.integers(0, 2**32, size=int(off[-1]), dtype=np.uint64).astype(np.uint32)
    return keys, off


def test_build_batch_rebases_offsets():
    rng = np.random.default_rng(0)
    jobs = [make_job(rng, 5) for _ in range(3)]

    class J:
        def __init__(self, k, o):
            self.keys, self.offsets = k, o
            self.nkeys = k.size

    keys, off, starts = build_batch([J(k, o) for k, o in jobs])
    assert keys.size == sum(k.size for k, _ in jobs) == off[-1]
    assert (np.diff(off) >= 0).all()
    assert off.size == sum(o.size - 1 for _, o in jobs) + 1
    for i, (k, o) in enumerate(jobs):
        assert (keys[starts[i]:starts[i + 1]] == k).all()


def test_results_match_oracle_and_accounting():
    rng = np.random.default_rng(1)
    ex = FakeExecutor(slots=2, service_s=0.002)
    jobs = [make_job(rng) for _ in range(40)]
    with SortServer(ex, hbm_budget=1 << 30, max_batch_jobs=4) as srv:
        hs = [srv.submit(k, o) for k, o in jobs]
        for h in hs:
            h.wait(30)
    for (k, o), h in zip(jobs, hs):
        want, _ = oracle.sort_segments(k, o)
        assert (h.result == want).all()
        assert h.completion >= h.admitted >= h.arrival
    st = srv.stats()
    assert st["jobs"] == 40 and st["latency_ms"]["p99"] >= st["latency_ms"]["p50"] > 0
    assert st["batches"] < 40, "queued jobs must be coalesced into shared batches"
    assert ex.concurrent_max == 2, "both slots must be used concurrently"


def test_budget_is_never_exceeded_and_fifo_without_starvation():
    rng = np.random.default_rng(2)
    ex = FakeExecutor(slots=3, service_s=0.003)
    jobs = [make_job(rng) for _ in range(60)]
    need = [device_bytes(k.size, o.size - 1, 4) for k, o in jobs]
    budget = 3 * max(need)
    with SortServer(ex, hbm_budget=budget) as srv:
        hs = [srv.submit(k, o) for k, o in jobs]
        for h in hs:
            h.wait(30)
    assert srv.max_inflight_bytes <= budget
    # admission is in arrival order: batches hold increasing, contiguous job ids
    flat = [jid for b in srv.batches for jid in b]
    assert flat == sorted(flat) == list(range(60))
    adm = [h.admitted for h in hs]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_job_larger_than_budget_is_rejected():
    ex = FakeExecutor()
    srv = SortServer(ex, hbm_budget=1000)
    with pytest.raises(AdmissionError):
        srv.submit(np.zeros(1000, np.uint32), np.array([0, 1000], np.int32))


def test_continuous_batching_admits_while_busy():
    """Jobs arriving while a batch runs are served by later batches, not after a drain."""
    rng = np.random.default_rng(3)
    ex = FakeExecutor(slots=1, service_s=0.02)
    with SortServer(ex, hbm_budget=1 << 30) as srv:
        first = srv.submit(*make_job(rng))
        time.sleep(0.005)  # first batch is running
        later = [srv.submit(*make_job(rng)) for _ in range(5)]
        for h in [first] + later:
            h.wait(30)
    assert first.batch_id == 0
    assert len({h.batch_id for h in later}) == 1 and later[0].batch_id == 1


def test_executor_failure_fails_jobs_and_keeps_serving():
    rng = np.random.default_rng(4)
    ex = FakeExecutor(slots=1, service_s=0.001, fail_on=1)
    with SortServer(ex, hbm_budget=1 << 30) as srv:
        bad = srv.submit(*make_job(rng))
        with pytest.raises(RuntimeError):
            bad.wait(30)
        good = srv.submit(*make_job(rng))
        good.wait(30)
    assert good.error is None


def test_concurrent_clients():
    rng = np.random.default_rng(5)
    jobs = [make_job(rng, 50) for _ in range(32)]
    ex = FakeExecutor(slots=2, service_s=0.001)
    out = {}
    with SortServer(ex, hbm_budget=1 << 30) as srv:
        def client(lo):
            for i in range(lo, lo + 8):
                out[i] = srv.submit(*jobs[i])
        ts = [threading.Thread(target=client, args=(8 * t,)) for t in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        for h in out.values():
            h.wait(30)
    for i, (k, o) in enumerate(jobs):
        assert (out[i].result == oracle.sort_segments(k, o)[0]).all()


def test_latency_counts_from_scheduled_arrival():
    """A client that submits late (behind its schedule) sees that delay in the
    job's latency: no coordinated omission."""
    rng = np.random.default_rng(11)
    ex = FakeExecutor(slots=2, service_s=0.001)
    k, o = make_job(rng, 5)
    with SortServer(ex) as srv:
        sched = time.monotonic() - 0.050  # the job was due 50 ms ago
        j = srv.submit(k, o, arrival=sched)
        j.wait(10)
    assert j.latency >= 0.050
    assert j.arrival == sched and j.queued >= sched + 0.050


def test_admission_counts_every_copy_the_executor_makes():
    """An executor that keeps two copies of a job's keys is charged for both."""
    rng = np.random.default_rng(12)
    k, o = make_job(rng, 5)

    class TwoCopies(FakeExecutor):
        def admission_bytes(self, job):
            return device_bytes(job.nkeys, job.nseg, self.key_bytes, 2)

    one = device_bytes(k.size, o.size - 1, 4, 1)
    two = device_bytes(k.size, o.size - 1, 4, 2)
    assert two - one == 4 * k.size
    ex = TwoCopies(slots=2, service_s=0.01)
    with SortServer(ex, hbm_budget=two + one // 2) as srv:  # room for one job's two copies only
        hs = [srv.submit(k, o) for _ in range(3)]
        for h in hs:
            h.wait(10)
    assert srv.max_inflight_bytes <= two + one // 2
    assert max(len(b) for b in srv.batches) == 1
    with pytest.raises(AdmissionError):
        SortServer(TwoCopies(), hbm_budget=two - 1).submit(k, o)


def test_batching_window_coalesces_jobs():
    """With a window, jobs that arrive while a batch runs wait for companions
    and leave in fewer, larger batches."""
    rng = np.random.default_rng(13)
    pool = [make_job(rng, 5) for _ in range(4)]

    def run(window):
        ex = FakeExecutor(slots=2, service_s=0.004)
        with SortServer(ex, max_batch_jobs=8, batch_window_s=window) as srv:
            hs = []
            for i in range(24):
                hs.append(srv.submit(*pool[i % 4]))
                time.sleep(0.0005)
            for h in hs:
                h.wait(10)
        return srv.stats()["mean_jobs_per_batch"]

    assert run(0.003) > run(0.0)
