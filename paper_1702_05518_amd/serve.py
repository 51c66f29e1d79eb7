"""Continuous-batching server for sampling jobs (orchestration over the C ABI).

A job asks for `nsweeps` chromatic Gibbs sweeps (Sec. 2.3, Algorithm 1, with
the Sec. 3.1 hyperparameter draws) of one chain on one graph and returns the
posterior mean and variance.  The server keeps every admitted chain resident
on the device and advances all active chains together, `step_sweeps` sweeps
at a time, through one gmrf batch (shared launches).  Between steps it
retires finished jobs and admits waiting ones while their device footprint
(gmrf_chain_footprint) fits the memory budget and a slot is free, so a job
that arrives while others run starts at the next step boundary.

Every job's chain is keyed by its own (seed, instance), never by its slot,
and the batch launches compute each chain exactly as a standalone sweep, so a
job's result is the same alone and in any mix, bit for bit.

All sampling runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import gmrf


@dataclasses.dataclass
class Job:
    job_id: int
    graph: "gmrf.Graph"
    y: np.ndarray
    seed: int
    instance: int
    nsweeps: int = 1000
    arrival: float = 0.0              # seconds after the start of the run
    precision: int = gmrf.FP32_ACC64
    # filled by the server
    chain: "gmrf.Chain | None" = None
    done: int = 0
    t_admit: float = float("nan")
    t_finish: float = float("nan")
    mean: "np.ndarray | None" = None
    var: "np.ndarray | None" = None

    @property
    def latency(self) -> float:
        return self.t_finish - self.arrival

    @property
    def sites(self) -> int:
        return self.graph.n


def chain_bytes(graph: "gmrf.Graph", precision: int) -> int:
    """Device bytes a job occupies while resident (its chain workspace)."""
    return int(gmrf.lib().gmrf_chain_footprint(graph.handle, precision))


class Server:
    """Admission by footprint, resident chains, one batch of shared launches
    per step.  `budget_bytes` bounds the summed chain footprints of the
    active jobs; `max_active` bounds their number.

    With `overlap`, the host work between steps (chain creation, the batch
    rebuild, reading finished jobs' results) runs while the device sweeps
    the steps already queued, at most `ahead` of them: chains and batches
    are created on a side stream, so their uploads wait for nothing the
    sweeps do; a job leaves the active set when its last step is queued,
    and its mean and variance are read on the side stream once the event
    after that step has completed; every chain or batch that queued sweeps
    still read stays referenced until their event has completed.  Without
    it, the server synchronises after every step."""

    def __init__(self, budget_bytes: int, step_sweeps: int = 10, max_active: int = 1024,
                 capture: bool = False, overlap: bool = False, ahead: int = 2):
        self.budget = int(budget_bytes)
        self.step_sweeps = int(step_sweeps)
        self.max_active = int(max_active)
        self.capture = capture
        self.overlap = overlap
        self.ahead = max(1, int(ahead))
        self.waiting: collections.deque = collections.deque()
        self.active: list = []
        self.finished: list = []
        self.used = 0
        self._batch = None
        self._batch_key = None
        self._side = None
        self._inflight: collections.deque = collections.deque()   # (event, objects kept alive)
        self._retiring: list = []                                 # (job, event of its last step)
        self.steps = 0
        self.rebuilds = 0

    # queue --------------------------------------------------------------
    def submit(self, job: Job):
        if job.nsweeps % self.step_sweeps:
            raise ValueError("nsweeps must be a multiple of step_sweeps")
        if chain_bytes(job.graph, job.precision) > self.budget:
            raise ValueError(f"job {job.job_id} alone exceeds the memory budget")
        self.waiting.append(job)

    def _create_stream(self):
        """The stream chains and batches are created on."""
        if not self.overlap:
            return None
        if self._side is None:
            import torch

            self._side = torch.cuda.Stream()
        return self._side

    def _admit(self, now: float):
        while self.waiting and len(self.active) < self.max_active:
            job = self.waiting[0]
            need = chain_bytes(job.graph, job.precision)
            if self.used + need > self.budget:
                break
            self.waiting.popleft()
            job.chain = gmrf.Chain(job.graph, job.y, precision=job.precision, seed=job.seed,
                                   instance=job.instance, stream=self._create_stream())
            job.t_admit = now
            self.used += need
            self.active.append(job)

    def _finish(self, job: Job, now: float, stream=None):
        job.mean, job.var, _ = job.chain.posterior_stats(stream=stream)
        job.t_finish = now
        self.used -= chain_bytes(job.graph, job.precision)
        job.chain = None
        self.finished.append(job)

    def _retire(self, now: float):
        keep = []
        for job in self.active:
            if job.done >= job.nsweeps:
                self._finish(job, now)         # posterior_stats synchronises the stream
            else:
                keep.append(job)
        self.active = keep

    def _collect(self, clock, wait: bool = False):
        """Overlap: read the results of jobs whose last step has completed
        (with `wait`, of every retiring job)."""
        keep = []
        for job, ev in self._retiring:
            if wait:
                ev.synchronize()
            if ev.query():
                side = self._create_stream()
                side.wait_event(ev)
                self._finish(job, clock(), stream=side)
            else:
                keep.append((job, ev))
        self._retiring = keep
        while self._inflight and self._inflight[0][0].query():
            self._inflight.popleft()

    # work ---------------------------------------------------------------
    def step(self, clock):
        """Admit, advance every active chain by step_sweeps sweeps, retire."""
        if self.overlap:
            return self._step_overlap(clock)
        self._admit(clock())
        if not self.active:
            return False
        key = tuple(j.job_id for j in self.active)
        if key != self._batch_key:
            self._batch = gmrf.Batch([j.chain for j in self.active])
            self._batch_key = key
            self.rebuilds += 1
        self._batch.sweep(self.step_sweeps, hyper=True, capture=self.capture)
        for job in self.active:
            job.done += self.step_sweeps
        self.steps += 1
        if any(j.done >= j.nsweeps for j in self.active):
            self._retire(clock())          # posterior_stats synchronises the stream
            self._batch, self._batch_key = None, None
        return True

    def _step_overlap(self, clock):
        import torch

        self._collect(clock)
        self._admit(clock())
        if not self.active:
            return False
        key = tuple(j.job_id for j in self.active)
        if key != self._batch_key:
            self._batch = gmrf.Batch([j.chain for j in self.active], stream=self._create_stream())
            self._batch_key = key
            self.rebuilds += 1
        main = torch.cuda.current_stream()
        self._batch.sweep(self.step_sweeps, hyper=True, capture=self.capture, stream=main)
        ev = torch.cuda.Event()
        ev.record(main)
        self._inflight.append((ev, (self._batch, [j.chain for j in self.active])))
        for job in self.active:
            job.done += self.step_sweeps
        self.steps += 1
        done = [j for j in self.active if j.done >= j.nsweeps]
        if done:
            self._retiring.extend((j, ev) for j in done)
            self.active = [j for j in self.active if j.done < j.nsweeps]
        while len(self._inflight) > self.ahead:
            self._inflight[0][0].synchronize()
            self._collect(clock)
        return True

    def run(self, jobs, realtime: bool = True):
        """Serve `jobs` (sorted by arrival).  With realtime, job.arrival is a
        wall-clock offset and a job becomes visible only after it has arrived;
        otherwise every job is visible at once.  Returns wall seconds."""
        import torch

        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: 0.0)
        while pending or self.waiting or self.active or self._retiring:
            now = clock()
            while pending and (not realtime or pending[0].arrival <= now):
                self.submit(pending.popleft())
            if not self.step(clock):
                if self._retiring:
                    self._collect(clock, wait=not pending)
                if pending:
                    wait = pending[0].arrival - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.001 if self._retiring else 0.01))
                continue
            if realtime and not self.overlap:
                torch.cuda.current_stream().synchronize()
        self._collect(clock, wait=True)
        self._inflight.clear()
        return time.perf_counter() - t0


def serve_plain(jobs, precision: int = gmrf.FP64, realtime: bool = True):
    """The unbatched baseline: one job at a time in arrival order, each a
    standalone chain swept with plain launches."""
    import torch

    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for job in sorted(jobs, key=lambda j: j.arrival):
        if realtime:
            wait = job.arrival - clock()
            if wait > 0:
                time.sleep(wait)
        ch = gmrf.Chain(job.graph, job.y, precision=precision, seed=job.seed,
                        instance=job.instance)
        job.t_admit = clock()
        ch.sweep(job.nsweeps)
        job.mean, job.var, _ = ch.posterior_stats()
        torch.cuda.current_stream().synchronize()
        job.t_finish = clock()
        job.done = job.nsweeps
    return time.perf_counter() - t0


def latency_summary(jobs):
    lat = np.array([j.latency for j in jobs]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "jobs": len(jobs)}
