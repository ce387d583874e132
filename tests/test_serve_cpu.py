"""The serving scheduler on a fake backend with a virtual clock (CPU only):
admission by footprint, continuous batching, latency accounting, and
checkpoint / restore.  The fake backend does no physics; it only tracks how
many sweeps each job received."""
import hashlib

import numpy as np
import pytest

from paper_2502_18624_amd.serve import Job, Server, poisson_trace


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance_to(self, t):
        self.t = max(self.t, t)


class FakeBackend:
    """Footprint L^2/2 bytes; a sweep of L^2 updates costs L^2 / rate seconds."""

    def __init__(self, clock, rate=1e10):
        self.clock, self.rate = clock, rate
        self.calls = []

    def footprint(self, model, L):
        return L * L // 2

    def create(self, job):
        return {"job": job.job_id, "t": 0, "L": job.L, "seed": job.seed}

    def restore(self, job, packed, t):
        return {"job": job.job_id, "t": t, "L": job.L, "seed": job.seed}

    def group_sweep(self, handles, n, betas, Ds):
        self.calls.append([(h["job"], k) for h, k in zip(handles, n)])
        for h, k in zip(handles, n):
            h["t"] += k
        self.clock.t += sum(k * h["L"] ** 2 for h, k in zip(handles, n)) / self.rate

    def synchronize(self):
        pass

    def record(self):
        return self.clock.t

    def wait(self, ev):
        pass

    def elapsed(self, a, b):
        return b - a

    def finish(self, h, corr):
        return {"t": h["t"]}

    def packed(self, h):
        return np.frombuffer(hashlib.sha256(b"%d-%d" % (h["seed"], h["t"])).digest(), dtype=np.uint8)

    def free(self, h):
        h["freed"] = True


def make_server(budget=2**22, tick=0.001):
    clock = VirtualClock()
    be = FakeBackend(clock)
    return Server(backend=be, hbm_budget=budget, tick_seconds=tick, clock=clock, rate_guess=1e10), be


def test_every_job_finishes_with_its_sweeps():
    srv, be = make_server(budget=2**26)
    jobs = poisson_trace(60, rate_per_s=2000, L_log2=(6, 10), sweeps_log10=(1, 3))
    st = srv.run_trace(jobs)
    assert st["jobs"] == 60
    for j in srv.finished:
        assert j.done == j.sweeps and j.result["t"] == j.sweeps
        assert j.arrival <= j.admitted <= j.finished
    assert st["latency_p99_s"] >= st["latency_p50_s"] > 0
    assert srv.in_use == 0


def test_admission_respects_the_budget():
    srv, be = make_server(budget=3 * 512 * 512 // 2)        # room for three L = 512 jobs
    jobs = [Job(i, 0, 512, i, 0.4, 0.0, 50, arrival=0.0) for i in range(7)]
    srv.run_trace(jobs)
    assert max(len(c) for c in be.calls) == 3
    assert srv.peak_bytes <= srv.budget
    with pytest.raises(ValueError):
        srv.submit(Job(99, 0, 4096, 1, 0.4, 0.0, 1))       # larger than the whole budget


def test_first_fit_in_arrival_order():
    srv, be = make_server(budget=1024 * 1024 // 2 + 2 * 64 * 64 // 2)
    big = [Job(0, 0, 1024, 1, 0.4, 0.0, 400, arrival=0.0), Job(1, 0, 1024, 2, 0.4, 0.0, 10, arrival=0.0)]
    small = [Job(2, 0, 64, 3, 0.4, 0.0, 10, arrival=0.0), Job(3, 0, 64, 4, 0.4, 0.0, 10, arrival=0.0)]
    srv.run_trace(big + small)
    first = dict(be.calls[0])
    assert 0 in first and 1 not in first and 2 in first and 3 in first
    order = [j.job_id for j in sorted(srv.finished, key=lambda j: j.admitted)]
    assert order.index(1) > order.index(0)


def test_continuous_batching_admits_while_others_run():
    srv, be = make_server(budget=2**26)
    long_job = Job(0, 0, 1024, 1, 0.4, 0.0, 2000, arrival=0.0)
    late = Job(1, 1, 256, 2, 0.4, 0.5, 20, arrival=0.01)
    srv.run_trace([long_job, late])
    lj = next(j for j in srv.finished if j.job_id == 0)
    lt = next(j for j in srv.finished if j.job_id == 1)
    assert lt.admitted < lj.finished                 # joined the running batch
    assert lt.finished < lj.finished                 # and left it early
    assert any(len(c) == 2 for c in be.calls)


def test_checkpoint_restore_gives_the_same_results():
    jobs_a = poisson_trace(25, rate_per_s=500, L_log2=(6, 9), sweeps_log10=(1, 3), seed=9)
    jobs_b = poisson_trace(25, rate_per_s=500, L_log2=(6, 9), sweeps_log10=(1, 3), seed=9)
    srv, _ = make_server(budget=2**26)
    srv.run_trace(jobs_a)
    ref = {j.job_id: j.digest for j in srv.finished}
    srv1, be1 = make_server(budget=2**26)
    srv1.run_trace(jobs_b, stop_after=5)
    state = srv1.checkpoint()
    srv2, be2 = make_server(budget=2**26)
    be2.clock.t = be1.clock.t
    srv2.t0 = srv1.t0
    srv2.restore(state)
    done = {j.job_id for j in state["finished"]} | {j.job_id for j, _, _ in state["live"]}
    rest = [j for j in jobs_b if j.job_id not in done and j not in state["pending"]]
    srv2.run_trace(rest)
    got = {j.job_id: j.digest for j in srv2.finished}
    assert got == ref


def test_ticks_in_flight_are_bounded_and_each_waited_once():
    clock = VirtualClock()
    be = FakeBackend(clock)
    waited = []
    be.wait = waited.append
    srv = Server(backend=be, hbm_budget=2**26, tick_seconds=0.001, clock=clock, rate_guess=1e10, depth=2)
    depths = []
    tick = srv.tick

    def counting_tick():
        r = tick()
        depths.append(len(srv._inflight))
        return r

    srv.tick = counting_tick
    st = srv.run_trace(poisson_trace(30, rate_per_s=2000, L_log2=(6, 9), sweeps_log10=(1, 2.5)))
    assert st["jobs"] == 30 and srv.ticks > 5
    assert max(depths) <= 2
    assert len(waited) == srv.ticks                  # one wait per tick, after later ticks were queued
    assert srv.in_use == 0 and not srv._inflight and not srv._retiring


def test_retirement_runs_beside_later_ticks():
    """The first job's retirement blocks until two more ticks have been
    queued: with retirement on the main thread this would never happen."""
    import threading
    clock = VirtualClock()
    be = FakeBackend(clock)
    go = threading.Event()
    calls = []
    sweep = be.group_sweep

    def group_sweep(handles, n, betas, Ds):
        sweep(handles, n, betas, Ds)
        calls.append(len(handles))
        if len(calls) >= 3:
            go.set()

    finish = be.finish

    def finish_after_two_more_ticks(h, corr):
        if h["job"] == 0:
            assert go.wait(timeout=10), "later ticks were not queued while a job retired"
        return finish(h, corr)

    be.group_sweep = group_sweep
    be.finish = finish_after_two_more_ticks
    srv = Server(backend=be, hbm_budget=2**26, tick_seconds=0.001, clock=clock, rate_guess=1e10, max_chunk=1)
    jobs = [Job(0, 0, 64, 1, 0.4, 0.0, 1, arrival=0.0), Job(1, 0, 64, 2, 0.4, 0.0, 6, arrival=0.0)]
    srv.run_trace(jobs)
    done = {j.job_id: j for j in srv.finished}
    assert set(done) == {0, 1} and done[0].result["t"] == 1 and done[1].result["t"] == 6
    assert len(calls) >= 3
