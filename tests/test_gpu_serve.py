"""Served jobs on the GPU: every job's final lattice and measurement are the
same alone and in the mix (bit-exact), whatever ticks and chunks the server
gave it; a checkpoint taken mid-trace and restored in a fresh server gives
the same results."""
import hashlib
import math

import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2


@pytest.fixture(scope="module")
def mcl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_18624_amd as m
    m.lib()
    return m


def _trace(seed):
    from paper_2502_18624_amd.serve import poisson_trace
    return poisson_trace(14, rate_per_s=400.0, seed=seed, L_log2=(6, 9), sweeps_log10=(0.7, 1.8))


def test_served_results_equal_solo_runs(mcl):
    from paper_2502_18624_amd.serve import Server
    print("serve mix vs solo", flush=True)
    jobs = _trace(4)
    srv = Server(hbm_budget=40 * 2**20, tick_seconds=0.0005, max_chunk=7)
    st = srv.run_trace(jobs)
    assert st["jobs"] == len(jobs) and st["ticks"] > 3
    assert srv.peak_live >= 2                                  # jobs really shared ticks
    for j in srv.finished:
        lat = mcl.Lattice(j.model, j.L, j.seed)
        lat.sweep(j.sweeps, j.beta, j.D)
        m = lat.measure(j.corr)
        assert hashlib.sha256(lat.read_packed().tobytes()).hexdigest() == j.digest, j
        assert (m["B"], m["M"], m["Q"], m["t"]) == (j.result["B"], j.result["M"], j.result["Q"], j.sweeps)
    # and one of them against the oracle
    j = min(srv.finished, key=lambda j: j.L * j.L * j.sweeps)
    s = oracle.init(j.model, j.L, j.seed)
    oracle.sweep(s, j.model, j.seed, 0, j.sweeps, j.beta, j.D)
    om = oracle.measure(s)
    assert (om["B"], om["M"], om["Q"]) == (j.result["B"], j.result["M"], j.result["Q"])


def test_serve_checkpoint_restore(mcl):
    from paper_2502_18624_amd.serve import Server
    print("serve checkpoint/restore", flush=True)
    ref = Server(hbm_budget=40 * 2**20, tick_seconds=0.0005, max_chunk=5)
    ref.run_trace(_trace(11))
    want = {j.job_id: j.digest for j in ref.finished}
    jobs = _trace(11)
    a = Server(hbm_budget=40 * 2**20, tick_seconds=0.0005, max_chunk=5)
    a.run_trace([j for j in jobs], stop_after=4)
    state = a.checkpoint()
    for j, _, _ in state["live"]:                              # drop the device state
        a.backend.free(j.handle)
        j.handle = None
    b = Server(hbm_budget=40 * 2**20, tick_seconds=0.0005, max_chunk=5)
    b.t0 = a.t0
    b.restore(state)
    seen = {j.job_id for j in state["finished"]} | {j.job_id for j, _, _ in state["live"]}
    seen |= {j.job_id for j in state["pending"]}
    b.run_trace([j for j in jobs if j.job_id not in seen])
    got = {j.job_id: j.digest for j in b.finished}
    assert got == want
