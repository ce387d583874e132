"""Sweeps of small lattices replayed from a captured graph (32 sweeps per
replay, the sweep index read from a device word that the replay advances)
against the oracle, bit for bit: one call spanning several replays and a
remainder, calls split at arbitrary points, changes of temperature between
calls (new graphs, cached graphs, and more temperatures than the cache
holds), a restore at an arbitrary t up to the end of the sweep counter,
lattices on separate streams, the replay switched off and on, and a caller
that captures sweep() into a graph of its own."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2
PARAMS = {0: (BETA_C, 0.0), 1: (1 / 1.4, 1.0), 2: (BETA_C, 0.0)}


@pytest.fixture(scope="module")
def mcl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_18624_amd as m
    m.lib()
    return m


@pytest.fixture
def replay(monkeypatch):
    monkeypatch.setenv("MCL_SWEEP_GRAPH", "1")


def _oracle(model, L, seed, calls, start=None, t0=0):
    """The oracle through a sequence of (n, beta, D) calls from t0."""
    s = oracle.init(model, L, seed) if start is None else start.copy()
    t = t0
    for n, beta, D in calls:
        oracle.sweep(s, model, seed, t, n, beta, D, nthreads=8)
        t += n
    return s


@pytest.mark.parametrize("model", [0, 1, 2])
def test_one_call_spans_replays_and_remainder(mcl, replay, model):
    print("graph: one call", model, flush=True)
    L, seed, n = 256, 2101 + model, 69                  # two replays and 5 direct sweeps
    beta, D = PARAMS[model]
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, beta, D)
    assert lat.t == n
    assert np.array_equal(lat.read(), _oracle(model, L, seed, [(n, beta, D)]))


@pytest.mark.parametrize("model", [0, 1, 2])
def test_split_calls_and_temperature_changes(mcl, replay, model):
    """Calls of 40, 33, 64 and 35 sweeps alternating two temperatures: the
    second temperature captures a second graph, the return to the first
    replays the cached one with the device word set to the new t."""
    print("graph: split calls", model, flush=True)
    L, seed = 256, 2111 + model
    beta, D = PARAMS[model]
    beta2 = beta * 1.25
    calls = [(40, beta, D), (33, beta2, D), (64, beta, D), (35, beta2, D), (3, beta, D)]
    lat = mcl.Lattice(model, L, seed)
    for n, b, d in calls:
        lat.sweep(n, b, d)
    assert np.array_equal(lat.read(), _oracle(model, L, seed, calls))


def test_more_temperatures_than_the_cache(mcl, replay):
    """Six temperatures in turn (the per-lattice cache keeps four graphs),
    then the first again: evicted graphs are captured anew."""
    print("graph: cache eviction", flush=True)
    L, seed = 256, 2121
    betas = [BETA_C * f for f in (0.6, 0.8, 1.0, 1.2, 1.5, 2.0)]
    calls = [(32, b, 0.0) for b in betas] + [(32, betas[0], 0.0), (32, betas[5], 0.0)]
    lat = mcl.Lattice(mcl.ISING, L, seed)
    for n, b, d in calls:
        lat.sweep(n, b, d)
    assert np.array_equal(lat.read(), _oracle(0, L, seed, calls))


@pytest.mark.parametrize("model", [0, 1, 2])
def test_restore_near_the_end_of_the_counter(mcl, replay, model):
    """A state written at t = 2^32 - 69, then 69 sweeps (the last allowed):
    the device word runs up to 2^32 - 5 and the remainder is direct."""
    print("graph: end of counter", model, flush=True)
    L, seed = 256, 2131 + model
    beta, D = PARAMS[model]
    rng = np.random.default_rng(model)
    vals = [-1, 0, 1] if model == 1 else [-1, 1]
    s0 = rng.choice(vals, size=(L, L)).astype(np.int8)
    t0 = 2**32 - 69
    lat = mcl.Lattice(model, L, seed)
    lat.write(s0, t0)
    lat.sweep(69, beta, D)
    assert lat.t == 2**32
    assert np.array_equal(lat.read(), _oracle(model, L, seed, [(69, beta, D)], start=s0, t0=t0))


def test_replay_on_and_off_agree(mcl, monkeypatch):
    """The same 70 sweeps at L = 1024 with the replay switched off and on,
    for the three models: identical lattices, equal to the oracle."""
    print("graph: on/off", flush=True)
    for model in (0, 1, 2):
        beta, D = PARAMS[model]
        got = []
        for flag in ("0", "1"):
            monkeypatch.setenv("MCL_SWEEP_GRAPH", flag)
            lat = mcl.Lattice(model, 1024, 2141 + model)
            lat.sweep(70, beta, D)
            got.append(lat.read())
            lat.free()
        assert np.array_equal(got[0], got[1]), model
        assert np.array_equal(got[1], _oracle(model, 1024, 2141 + model, [(70, beta, D)])), model


def test_replays_on_separate_streams(mcl, replay):
    """Three lattices on their own streams, replays queued interleaved:
    each device word belongs to its lattice, each result equals the oracle."""
    import torch
    print("graph: streams", flush=True)
    streams = [torch.cuda.Stream() for _ in range(3)]
    specs = [(0, 512, 2151), (1, 256, 2152), (2, 512, 2153)]
    lats = [mcl.Lattice(m, L, sd, stream=st) for (m, L, sd), st in zip(specs, streams)]
    for _ in range(2):
        for lat, (m, L, sd) in zip(lats, specs):
            lat.sweep(33, *PARAMS[m])
    torch.cuda.synchronize()
    for lat, (m, L, sd) in zip(lats, specs):
        assert lat.t == 66
        assert np.array_equal(lat.read(), _oracle(m, L, sd, [(66, *PARAMS[m])])), m


def test_free_with_replays_queued_then_reuse(mcl, replay):
    """A handle freed right after queueing replays (the free waits for
    them), then a new handle on the same device buffer: its graphs are its
    own and its run equals the oracle."""
    print("graph: free and reuse", flush=True)
    L, beta = 512, BETA_C
    a = mcl.Lattice(mcl.ISING, L, 2161)
    a.sweep(96, beta)
    mem = a.mem
    a.free()
    b = mcl.Lattice(mcl.ISING, L, 2162, mem=mem)
    b.sweep(64, beta)
    assert np.array_equal(b.read(), _oracle(0, L, 2162, [(64, beta, 0.0)]))
    b.free()


@pytest.mark.parametrize("model", [0, 2])
def test_caller_captures_sweeps(mcl, replay, model):
    """A caller captures 40 sweeps of a handle on its own stream into a
    torch CUDA graph (sweep() then queues plain launches, even with the
    replay forced on) and replays it three times, with eager work and a
    synchronisation between replays: each replay repeats sweeps t = 0..39
    and matches the oracle applied to the previous state."""
    import torch
    print("graph: caller capture", model, flush=True)
    L, seed = 256, 2171 + model
    beta, D = PARAMS[model]
    st = torch.cuda.Stream()
    lat = mcl.Lattice(model, L, seed, stream=st)
    want = lat.read()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        lat.sweep(40, beta, D)
    assert lat.t == 40
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        want = _oracle(model, L, seed, [(40, beta, D)], start=want)
        assert np.array_equal(lat.read(), want), k
        x = torch.ones(4096, device="cuda")
        assert float((x + 1.0).sum()) == 8192.0             # eager work between replays
