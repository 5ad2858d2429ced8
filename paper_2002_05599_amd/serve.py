"""Continuous-batching sort service on one GPU.

Clients submit sort jobs -- each a ragged batch of segments (keys + CSR
offsets starting at 0) -- at any time.  A scheduler thread

  * admits jobs in arrival order while the device bytes of everything in
    flight stay within an HBM budget -- every copy the executor makes of a
    job counts (a job larger than the whole budget is rejected at
    submission; the oldest waiting job blocks younger ones, so no job
    starves);
  * coalesces the admitted jobs into one device batch (keys concatenated,
    offsets rebased) as soon as an execution slot is free, so jobs arriving
    while others run are picked up by the next batch (continuous batching);
    with a batching window, a batch that could still take more jobs waits up
    to that long for them while another batch is running;
  * runs each batch on its own slot -- a HIP stream with its own pinned
    staging buffers -- as host-to-device copy, one ``segmented_sort`` call
    and device-to-host copy, so the copies and sorts of several batches
    overlap on the device (the library keeps separate working memory per
    stream);
  * completes each job when its batch's event has fired, recording latency
    = completion time - arrival time on the host's monotonic clock, where
    the arrival time is the job's scheduled arrival when the client gives
    one (an open-loop client that falls behind its schedule then shows the
    delay in the latency instead of hiding it).

Results are bit-identical whether a job runs alone or inside a mixed batch:
segments are sorted independently and a batch only concatenates them.

The executor is pluggable: ``GpuExecutor`` drives the library; tests swap in
a host-only executor to check admission, ordering and accounting without a
GPU.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


class AdmissionError(ValueError):
    """A job can never fit the HBM budget."""


@dataclass
class Job:
    jid: int
    keys: np.ndarray
    offsets: np.ndarray
    arrival: float = 0.0
    admitted: float = 0.0
    completion: float = 0.0
    batch_id: int = -1
    result: Optional[np.ndarray] = None
    error: Optional[BaseException] = None
    done: threading.Event = field(default_factory=threading.Event)

    ready: object = None  # device jobs: event recorded on the submitting stream
    queued: float = 0.0   # when submit() queued it (time.monotonic())

    @property
    def nkeys(self) -> int:
        return int(self.keys.numel() if hasattr(self.keys, "numel") else self.keys.size)

    @property
    def nseg(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def latency(self) -> float:
        return self.completion - self.arrival

    def wait(self, timeout=None) -> np.ndarray:
        if not self.done.wait(timeout):
            raise TimeoutError(f"job {self.jid} not done")
        if self.error is not None:
            raise self.error
        return self.result


def device_bytes(nkeys: int, nseg: int, key_bytes: int, key_copies: int = 1) -> int:
    """HBM a job occupies while in flight: key_copies copies of its keys plus
    its offsets."""
    return key_copies * nkeys * key_bytes + (nseg + 1) * 4


def build_batch(jobs: List[Job]):
    """Concatenate jobs into one CSR batch: (keys, offsets, key_starts)."""
    sizes = [j.nkeys for j in jobs]
    starts = np.zeros(len(jobs) + 1, dtype=np.int64)
    np.cumsum(sizes, out=starts[1:])
    keys = np.concatenate([j.keys for j in jobs]) if jobs else np.zeros(0)
    parts = [(j.offsets[:-1].astype(np.int64) - int(j.offsets[0]) + starts[i]) for i, j in enumerate(jobs)]
    parts.append(np.array([starts[-1]], dtype=np.int64))
    offsets = np.concatenate(parts).astype(np.int32)
    return keys, offsets, starts


class GpuExecutor:
    """Runs batches through the library on ``slots`` HIP streams.

    Host jobs (numpy keys): the batch is assembled in pinned memory, copied to
    the device, sorted, and copied back; each job receives a numpy array.
    Device jobs (CUDA tensors): the batch is gathered on the device and each
    job receives a device tensor view of the sorted batch -- the data never
    leaves HBM.
    """

    def __init__(self, slots: int = 3, dtype=np.uint32, device: int = 0):
        import torch
        import paper_2002_05599_amd as ss
        self._torch = torch
        self._ss = ss
        self.dtype = np.dtype(dtype)
        self.device = torch.device("cuda", device)
        self.tdtype = {np.dtype(np.uint32): torch.uint32, np.dtype(np.int32): torch.int32,
                       np.dtype(np.uint64): torch.uint64, np.dtype(np.int64): torch.int64}[self.dtype]
        # default-priority streams only
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.busy = [False] * slots
        self.pinned_in = [None] * slots
        self.pinned_out = [None] * slots
        self.pinned_off = [None] * slots
        self.inflight = {}

    @property
    def key_bytes(self) -> int:
        return self.dtype.itemsize

    def admission_bytes(self, job) -> int:
        """HBM the job holds while its batch runs: a host job's keys are
        copied to the device once; a device job's keys are already resident
        and the batch gathers them into a second copy."""
        on_device = hasattr(job.keys, "is_cuda")
        return device_bytes(job.nkeys, job.nseg, self.key_bytes, 2 if on_device else 1)

    def free_slot(self) -> Optional[int]:
        for i, b in enumerate(self.busy):
            if not b:
                return i
        return None

    def _pinned(self, cache, slot, n, dtype):
        t = cache[slot]
        if t is None or t.numel() < n:
            t = self._torch.empty(max(n, 1024), dtype=dtype, pin_memory=True)
            cache[slot] = t
        return t

    def launch(self, slot: int, jobs: List[Job]):
        torch = self._torch
        starts = np.zeros(len(jobs) + 1, dtype=np.int64)
        np.cumsum([j.nkeys for j in jobs], out=starts[1:])
        n = int(starts[-1])
        parts = [j.offsets[:-1].astype(np.int64) - int(j.offsets[0]) + starts[i] for i, j in enumerate(jobs)]
        parts.append(np.array([n], dtype=np.int64))
        offsets = np.concatenate(parts).astype(np.int32)
        on_device = hasattr(jobs[0].keys, "is_cuda")
        hoff = self._pinned(self.pinned_off, slot, offsets.size, torch.int32)
        hoff[:offsets.size].numpy()[:] = offsets
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            do = torch.empty(offsets.size, dtype=torch.int32, device=self.device)
            do.copy_(hoff[:offsets.size], non_blocking=True)
            if on_device:
                for j in jobs:
                    if j.ready is not None:
                        stream.wait_event(j.ready)
                dk = torch.cat([j.keys for j in jobs]) if len(jobs) > 1 else jobs[0].keys.clone()
                hout = None
            else:
                hin = self._pinned(self.pinned_in, slot, n, self.tdtype)
                hout = self._pinned(self.pinned_out, slot, n, self.tdtype)
                hv = hin[:n].numpy()
                for i, j in enumerate(jobs):
                    hv[starts[i]:starts[i + 1]] = j.keys
                dk = torch.empty(n, dtype=self.tdtype, device=self.device)
                dk.copy_(hin[:n], non_blocking=True)
            self._ss.segmented_sort(dk, do, stream=stream)
            if hout is not None:
                hout[:n].copy_(dk, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.busy[slot] = True
        self.inflight[slot] = (ev, dk, do, hout, starts)

    def device_rate(self, pool, batch_jobs: int, reps: int = 3) -> float:
        """Jobs per second the device sustains on ``pool`` (a list of (keys,
        offsets) jobs, all on the device or all on the host) when it is
        served in batches of ``batch_jobs`` consecutive jobs back to back on
        one stream: the median over ``reps`` passes of HIP-event time, so the
        figure does not depend on how fast the host thread schedules."""
        torch = self._torch
        stream = self.streams[0]
        batches = [pool[i:i + batch_jobs] for i in range(0, len(pool), batch_jobs)]
        staged = []
        for b in batches:
            jobs = [Job(-1, k, np.ascontiguousarray(o, dtype=np.int32)) for k, o in b]
            starts = np.zeros(len(jobs) + 1, dtype=np.int64)
            np.cumsum([j.nkeys for j in jobs], out=starts[1:])
            parts = [j.offsets[:-1].astype(np.int64) - int(j.offsets[0]) + starts[i] for i, j in enumerate(jobs)]
            parts.append(np.array([int(starts[-1])], dtype=np.int64))
            off = torch.from_numpy(np.concatenate(parts).astype(np.int32)).pin_memory()
            keys = [j.keys if hasattr(j.keys, "is_cuda") else torch.from_numpy(j.keys).pin_memory() for j in jobs]
            staged.append((keys, off, int(starts[-1])))
        times = []
        for _ in range(reps):
            with torch.cuda.stream(stream):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for keys, off, n in staged:
                    do = off.to(self.device, non_blocking=True)
                    dk = torch.cat([k.to(self.device, non_blocking=True) for k in keys]) if len(keys) > 1 \
                        else keys[0].to(self.device, non_blocking=True).clone()
                    self._ss.segmented_sort(dk, do, stream=stream)
                    if not keys[0].is_cuda:
                        dk.to("cpu", non_blocking=True)
                e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        return len(pool) / float(np.median(times))

    def done(self, slot: int) -> bool:
        return self.inflight[slot][0].query()

    def result(self, slot: int):
        ev, dk, do, hout, starts = self.inflight.pop(slot)
        ev.synchronize()
        self.busy[slot] = False
        if hout is None:
            return [dk[starts[i]:starts[i + 1]] for i in range(len(starts) - 1)]
        out = hout[:int(starts[-1])].numpy()
        return [out[starts[i]:starts[i + 1]].copy() for i in range(len(starts) - 1)]


class SortServer:
    """Admission + continuous batching over an executor (see module docstring)."""

    def __init__(self, executor, hbm_budget: int = 16 << 30, max_batch_keys: int = 64 << 20,
                 max_batch_jobs: int = 256, poll_s: float = 20e-6, batch_window_s: float = 0.0):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch_keys = int(max_batch_keys)
        self.max_batch_jobs = int(max_batch_jobs)
        self.poll_s = poll_s
        self.batch_window_s = float(batch_window_s)
        self._lock = threading.Lock()
        self._cv = threading.Condition(self._lock)
        self._incoming = collections.deque()
        self._pending = collections.deque()
        self._inflight = {}  # slot -> (jobs, bytes, batch_id)
        self._inflight_bytes = 0
        self._next_jid = 0
        self._next_batch = 0
        self._stop = False
        self._thread = None
        self.completed: List[Job] = []
        self.batches: List[List[int]] = []
        self.max_inflight_bytes = 0
        self.max_concurrent_batches = 0

    # -- client side ----------------------------------------------------------
    def _job_bytes(self, job) -> int:
        f = getattr(self.ex, "admission_bytes", None)
        return f(job) if f is not None else device_bytes(job.nkeys, job.nseg, self.ex.key_bytes)

    def submit(self, keys, offsets: np.ndarray, arrival: Optional[float] = None) -> Job:
        """Queue a job: keys (numpy array, or a CUDA tensor already in HBM) and
        host int32 CSR offsets.  ``arrival``: the job's scheduled arrival on
        time.monotonic()'s clock (default: now); latency is measured from it.
        Returns a Job to wait on."""
        ready = None
        if hasattr(keys, "is_cuda") and keys.is_cuda:
            import torch
            ready = torch.cuda.Event()
            ready.record()
        else:
            keys = np.ascontiguousarray(keys)
        offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        now = time.monotonic()
        job = Job(-1, keys, offsets, arrival=now if arrival is None else float(arrival), ready=ready)
        need = self._job_bytes(job)
        if need > self.budget:
            raise AdmissionError(f"job needs {need} bytes of HBM, budget is {self.budget}")
        job.queued = now
        with self._cv:
            job.jid = self._next_jid
            self._next_jid += 1
            self._incoming.append(job)
            self._cv.notify()
        return job

    def start(self):
        self._thread = threading.Thread(target=self._run, name="sort-server", daemon=True)
        self._thread.start()
        return self

    def stop(self):
        """Stop after every submitted job has completed."""
        with self._cv:
            self._stop = True
            self._cv.notify()
        if self._thread:
            self._thread.join()

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    # -- scheduler ----------------------------------------------------------------
    def _admit_batch(self):
        """Pop the longest FIFO prefix of pending jobs that fits budget and batch limits."""
        jobs, nbytes, nkeys = [], 0, 0
        while self._pending and len(jobs) < self.max_batch_jobs:
            j = self._pending[0]
            need = self._job_bytes(j)
            if self._inflight_bytes + nbytes + need > self.budget:
                break
            if jobs and nkeys + j.nkeys > self.max_batch_keys:
                break
            jobs.append(self._pending.popleft())
            nbytes += need
            nkeys += j.nkeys
        return jobs, nbytes

    def _run(self):
        while True:
            with self._cv:
                while self._incoming:
                    self._pending.append(self._incoming.popleft())
                idle = not self._pending and not self._inflight
                if idle:
                    if self._stop:
                        return
                    self._cv.wait(0.01)
                    continue
            progressed = False
            # launch as many batches as slots and budget allow
            while self._pending:
                slot = self.ex.free_slot()
                if slot is None:
                    break
                if self._hold_for_window():
                    break
                jobs, nbytes = self._admit_batch()
                if not jobs:
                    break
                now = time.monotonic()
                bid = self._next_batch
                self._next_batch += 1
                for j in jobs:
                    j.admitted = now
                    j.batch_id = bid
                try:
                    self.ex.launch(slot, jobs)
                except BaseException as e:  # executor failure: fail the jobs, keep serving
                    for j in jobs:
                        j.error = e
                        j.completion = time.monotonic()
                        j.done.set()
                    continue
                self._inflight[slot] = (jobs, nbytes, bid)
                self._inflight_bytes += nbytes
                self.max_inflight_bytes = max(self.max_inflight_bytes, self._inflight_bytes)
                self.max_concurrent_batches = max(self.max_concurrent_batches, len(self._inflight))
                self.batches.append([j.jid for j in jobs])
                progressed = True
            # complete finished batches
            for slot in list(self._inflight):
                if not self.ex.done(slot):
                    continue
                jobs, nbytes, bid = self._inflight.pop(slot)
                try:
                    outs = self.ex.result(slot)
                    err = None
                except BaseException as e:
                    outs, err = None, e
                now = time.monotonic()
                for i, j in enumerate(jobs):
                    if err is None:
                        j.result = outs[i]
                    j.error = err
                    j.completion = now
                    j.done.set()
                    self.completed.append(j)
                self._inflight_bytes -= nbytes
                progressed = True
            if not progressed:
                time.sleep(self.poll_s)

    def _hold_for_window(self) -> bool:
        """With a batching window: while another batch runs, a batch that could
        take more jobs waits until its oldest job has queued for the window."""
        if self.batch_window_s <= 0 or not self._inflight or len(self._pending) >= self.max_batch_jobs:
            return False
        return time.monotonic() - self._pending[0].queued < self.batch_window_s

    # -- reporting -------------------------------------------------------------
    def stats(self):
        lat = np.array([j.latency for j in self.completed if j.error is None])
        if lat.size == 0:
            return {"jobs": 0}
        keys = sum(j.nkeys for j in self.completed)
        t0 = min(j.arrival for j in self.completed)
        t1 = max(j.completion for j in self.completed)
        return {
            "jobs": int(lat.size), "keys": int(keys), "span_s": t1 - t0,
            "keys_per_s": keys / (t1 - t0) if t1 > t0 else None,
            "latency_ms": {q: float(np.percentile(lat, p) * 1e3)
                           for q, p in (("p50", 50), ("p90", 90), ("p99", 99), ("max", 100))},
            "batches": len(self.batches),
            "mean_jobs_per_batch": float(np.mean([len(b) for b in self.batches])),
            "max_concurrent_batches": self.max_concurrent_batches,
            "max_inflight_bytes": self.max_inflight_bytes,
        }


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s, from 0) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def run_open_loop(server: SortServer, jobs, arrivals: np.ndarray):
    """Submit jobs[i % len(jobs)] at arrivals[i] (relative, seconds); wait for
    all.  Each job's latency counts from its scheduled arrival, so time the
    client spends behind schedule is part of it."""
    t0 = time.monotonic()
    handles = []
    for i, at in enumerate(arrivals):
        delay = t0 + at - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        k, off = jobs[i % len(jobs)]
        handles.append(server.submit(k, off, arrival=t0 + at))
    for h in handles:
        h.wait(timeout=600)
    return handles
