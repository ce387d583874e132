"""Serving loop: continuous batching of quench-simulation jobs.

A job is (model, L, seed, beta, D, sweeps): a lattice quenched from its T =
infinity sample and relaxed for `sweeps` checkerboard sweeps, then measured.
The server:

- admits arrived jobs in arrival order (first fit) while their device
  footprint (``mcl_query_bytes``) fits the HBM budget;
- keeps every admitted lattice and its sweep counter resident on the device;
- runs ticks: one ``group_sweep`` over all live jobs, each advancing by a
  chunk of sweeps sized so that a tick takes about ``tick_seconds``; jobs
  that arrive meanwhile join at the next tick (continuous batching);
- keeps up to ``depth`` ticks queued on the device: after queuing a tick it
  records an event and waits only for the event of the tick ``depth``
  before, so the host plans and queues the next tick while the device runs
  the current one (no device-wide synchronisation);
- retires finished jobs on a worker thread (final measurement, optional
  digest, memory freed) while the following ticks run; a job's memory
  returns to the budget when its retirement completes;
- records arrival -> admission -> completion times.

Because the draws are keyed by (seed, sweep, site), a job's result does not
depend on which other jobs shared its ticks or how its sweeps were chunked.
"""
from __future__ import annotations

import hashlib
import math
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from ._lib import CORR_NONE


@dataclass
class Job:
    job_id: int
    model: int
    L: int
    seed: int
    beta: float
    D: float
    sweeps: int
    arrival: float = 0.0                # seconds after the trace start
    corr: int = CORR_NONE               # correlation mode of the final measurement
    admitted: Optional[float] = None
    finished: Optional[float] = None
    done: int = 0                       # sweeps completed
    result: Optional[dict] = None
    digest: Optional[str] = None        # sha256 of the final packed lattice
    handle: object = field(default=None, repr=False)

    @property
    def updates(self) -> int:
        return self.L * self.L * self.sweeps


class LibraryBackend:
    """Jobs as library lattices on the current torch stream."""

    def __init__(self, device="cuda"):
        self.device = device

    def footprint(self, model, L):
        from .lattice import query_bytes
        return query_bytes(model, L) + 256

    def create(self, job):
        from .lattice import Lattice
        return Lattice(job.model, job.L, job.seed, device=self.device)

    def restore(self, job, packed, t):
        lat = self.create(job)
        lat.write_packed(packed, t)
        return lat

    def group_sweep(self, handles, n, betas, Ds):
        from .lattice import group_sweep
        group_sweep(handles, n, betas, Ds)

    def synchronize(self):
        import torch
        torch.cuda.synchronize()

    def record(self):
        """A timing event queued on the current stream."""
        import torch
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        return ev

    def wait(self, ev):
        ev.synchronize()

    def elapsed(self, a, b):
        """Seconds between two completed events."""
        return a.elapsed_time(b) * 1e-3

    def finish(self, handle, corr):
        return handle.measure(corr)

    def packed(self, handle):
        return handle.read_packed()

    def free(self, handle):
        handle.free()


class Server:
    def __init__(self, backend=None, hbm_budget=250e9, tick_seconds=0.02, max_chunk=256, clock=time.perf_counter,
                 rate_guess=2.0e12, keep_digest=True, depth=2, retire_thread=True):
        self.backend = backend or LibraryBackend()
        self.depth = max(1, int(depth))     # ticks queued on the device at most
        self._inflight = deque()            # (start event, end event, updates) of queued ticks
        self._retiring = []                 # (job, future or None) of jobs being retired
        self._pool = ThreadPoolExecutor(max_workers=1) if retire_thread else None
        self.budget = float(hbm_budget)
        self.tick_seconds = tick_seconds
        self.max_chunk = max_chunk
        self.clock = clock
        self.rate = rate_guess              # updates/s, refined from measured ticks
        self.keep_digest = keep_digest
        self.pending = []                   # arrived, not admitted (arrival order)
        self.live = []
        self.finished = []
        self.in_use = 0.0
        self.t0 = None
        self.ticks = 0
        self.peak_live = 0
        self.peak_bytes = 0.0

    # -- admission ---------------------------------------------------------
    def submit(self, job: Job):
        if self.backend.footprint(job.model, job.L) > self.budget:
            raise ValueError("job %d needs more than the whole HBM budget" % job.job_id)
        self.pending.append(job)

    def now(self):
        return self.clock() - self.t0

    def _admit(self):
        keep = []
        for job in self.pending:
            need = self.backend.footprint(job.model, job.L)
            if self.in_use + need <= self.budget:
                job.handle = self.backend.create(job)
                job.admitted = self.now()
                self.in_use += need
                self.live.append(job)
            else:
                keep.append(job)
        self.pending = keep
        self.peak_live = max(self.peak_live, len(self.live))
        self.peak_bytes = max(self.peak_bytes, self.in_use)

    # -- one tick ------------------------------------------------------------
    def _chunk(self):
        work = sum(j.L * j.L for j in self.live)
        if work == 0:
            return 1
        c = int(self.tick_seconds * self.rate / work)
        return max(1, min(self.max_chunk, c))

    def tick(self):
        """Queue one tick; wait for the tick `depth` before it; hand the jobs
        this tick completes to the retirement worker."""
        if not self.live:
            return 0
        chunk = self._chunk()
        n = [min(chunk, j.sweeps - j.done) for j in self.live]
        ev0 = self.backend.record()
        self.backend.group_sweep([j.handle for j in self.live], n, [j.beta for j in self.live],
                                 [j.D for j in self.live])
        ev1 = self.backend.record()
        upd = sum(k * j.L * j.L for k, j in zip(n, self.live))
        self._inflight.append((ev0, ev1, upd))
        for k, j in zip(n, self.live):
            j.done += k          # queued: later ticks and the final measurement follow in stream order
        self.ticks += 1
        self._retire()
        while len(self._inflight) > self.depth:
            self._complete_oldest()
        self._collect(block=False)
        return upd

    def _complete_oldest(self):
        ev0, ev1, upd = self._inflight.popleft()
        self.backend.wait(ev1)
        el = self.backend.elapsed(ev0, ev1)
        if el > 0 and upd > 0:
            self.rate = 0.7 * self.rate + 0.3 * (upd / el)

    def _finish_job(self, j):
        j.result = self.backend.finish(j.handle, j.corr)      # waits for the job's last tick
        if self.keep_digest:
            j.digest = hashlib.sha256(np.asarray(self.backend.packed(j.handle)).tobytes()).hexdigest()
        j.finished = self.now()
        self.backend.free(j.handle)
        j.handle = None
        return j

    def _retire(self):
        still = []
        for j in self.live:
            if j.done >= j.sweeps:
                if self._pool is None:
                    self._finish_job(j)
                    self._retiring.append((j, None))
                else:
                    self._retiring.append((j, self._pool.submit(self._finish_job, j)))
            else:
                still.append(j)
        self.live = still

    def _collect(self, block):
        """Account the retirements that have completed (all of them if block)."""
        keep = []
        for j, fut in self._retiring:
            if fut is not None and not block and not fut.done():
                keep.append((j, fut))
                continue
            if fut is not None:
                fut.result()                                  # re-raises a failed retirement
            self.in_use -= self.backend.footprint(j.model, j.L)
            self.finished.append(j)
        self._retiring = keep

    def drain(self):
        """Wait for every queued tick and retirement."""
        while self._inflight:
            self._complete_oldest()
        self._collect(block=True)

    # -- a whole trace -------------------------------------------------------
    def run_trace(self, jobs, stop_after=None):
        """Feed `jobs` at their arrival times (seconds after the start) and run
        until all have finished (or `stop_after` ticks).  Returns stats."""
        arrivals = sorted(jobs, key=lambda j: j.arrival)
        if self.t0 is None:
            self.t0 = self.clock()
        i = 0
        while i < len(arrivals) or self.pending or self.live or self._retiring:
            now = self.now()
            while i < len(arrivals) and arrivals[i].arrival <= now:
                self.submit(arrivals[i])
                i += 1
            self._admit()
            if self.live:
                self.tick()
                if stop_after is not None and self.ticks >= stop_after:
                    break
            elif self._retiring or self._inflight:
                # nothing to sweep: let the queued work and retirements finish
                while self._inflight:
                    self._complete_oldest()
                self._collect(block=not self.pending and i >= len(arrivals))
                if self._retiring:
                    time.sleep(0.0005)
            elif i < len(arrivals):
                # idle until the next arrival
                if hasattr(self.clock, "advance_to"):
                    self.clock.advance_to(self.t0 + arrivals[i].arrival)
                else:
                    time.sleep(max(0.0, min(arrivals[i].arrival - self.now(), 0.05)))
            elif self.pending:
                raise RuntimeError("jobs pending with nothing live or retiring: the budget cannot hold them")
        self.drain()
        return self.stats()

    def stats(self):
        done = self.finished
        if not done:
            return {"jobs": 0}
        lat = np.array([j.finished - j.arrival for j in done])
        wait = np.array([j.admitted - j.arrival for j in done])
        end = max(j.finished for j in done)
        start = min(j.arrival for j in done)
        upd = float(sum(j.updates for j in done))
        return {
            "jobs": len(done),
            "updates": upd,
            "updates_per_ns": upd / max(end - start, 1e-12) / 1e9,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "queue_wait_p50_s": float(np.percentile(wait, 50)),
            "queue_wait_p99_s": float(np.percentile(wait, 99)),
            "ticks": self.ticks,
            "peak_live_jobs": self.peak_live,
            "peak_bytes": self.peak_bytes,
        }

    # -- checkpoint / restore --------------------------------------------------
    def checkpoint(self):
        """Host copy of every live job (packed lattice and sweep counter) and
        the queue; the device state can then be dropped."""
        self.drain()
        self.backend.synchronize()
        live = []
        for j in self.live:
            live.append((j, np.asarray(self.backend.packed(j.handle)).copy(), j.done))
        return {"live": live, "pending": list(self.pending), "finished": list(self.finished)}

    def restore(self, state):
        for j, packed, done in state["live"]:
            j.handle = self.backend.restore(j, packed, done)
            j.done = done
            self.in_use += self.backend.footprint(j.model, j.L)
            self.live.append(j)
        self.pending = list(state["pending"])
        self.finished = list(state["finished"])


def poisson_trace(n_jobs, rate_per_s=200.0, seed=4, L_log2=(10, 15), sweeps_log10=(2, 4), t_frac=(0.5, 1.5),
                  D_choices=(0.0, 0.5, 1.0)):
    """Quench jobs with Poisson arrivals: exponential inter-arrival times of
    mean 1/rate, L = 64 round(2^U[a,b] / 64), sweeps = round(10^U[c,d]),
    T ~ U[t_frac] * T_c, D from D_choices (Blume-Capel), model 50/50."""
    rng = np.random.default_rng(seed)
    beta_c = math.log(1 + math.sqrt(2)) / 2
    t = 0.0
    jobs = []
    for i in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        L = int(64 * round(2 ** rng.uniform(*L_log2) / 64))
        L = max(L, 64)
        sweeps = int(round(10 ** rng.uniform(*sweeps_log10)))
        model = int(rng.integers(0, 2))
        T = float(rng.uniform(*t_frac)) / beta_c
        D = float(rng.choice(D_choices)) if model == 1 else 0.0
        jobs.append(Job(job_id=i, model=model, L=L, seed=int(rng.integers(1, 2**63)), beta=1.0 / T, D=D,
                        sweeps=sweeps, arrival=t))
    return jobs
