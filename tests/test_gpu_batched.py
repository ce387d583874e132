"""Batched path at the benchmark's replica mix, bit for bit.

The batched workload holds hundreds of replicas of L = 512 ... 8192 with
temperatures drawn around T_c and crystal fields in {0, 0.5, 1}.  Here a
sample of that mix -- 36 replicas, all three models, every size of the
workload -- runs through group_sweep with the tuning the autotuner picks for
it, and every replica's final lattice must equal its own plain sweep() run
(packed digest; the plain path is itself checked against the oracle by the
other tests).  The same holds with the work split over several calls of one
shape (plain launches, then a captured graph, then its replay), and for a
lattice too large for the batched launches, which the call sweeps on its
own."""
import hashlib
import math

import numpy as np
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


def _mix(n, seed):
    rng = np.random.default_rng(seed)
    specs = []
    sizes = [512, 1024, 2048, 4096, 8192]
    for i in range(n):
        model = i % 3
        L = sizes[i % len(sizes)] if i < len(sizes) * 3 else int(rng.choice(sizes))
        beta = 1.0 / (float(rng.uniform(0.5, 1.5)) / BETA_C)
        D = float(rng.choice([0.0, 0.5, 1.0])) if model == 1 else 0.0
        specs.append((model, L, 7000 + i, beta, D))
    return specs


def _digest(lat):
    return hashlib.sha256(lat.read_packed().tobytes()).hexdigest()


def _run_mix_against_plain(mcl, specs, seed):
    """Three calls of one shape (plain launches, then a captured graph, then
    its replay under graph tunings), then a new shape with some replicas
    idle; every replica's packed lattice against its own sweep() run."""
    rng = np.random.default_rng(seed)
    calls = [[int(rng.integers(1, 6)) for _ in specs] for _ in range(3)]   # one shape, three calls
    calls.append([int(rng.integers(0, 3)) for _ in specs])                  # a new shape, some idle
    lats = [mcl.Lattice(m, L, sd) for (m, L, sd, _, _) in specs]
    for n in calls:
        mcl.group_sweep(lats, n, [sp[3] for sp in specs], [sp[4] for sp in specs])
    for i, (lat, (m, L, sd, b, D)) in enumerate(zip(lats, specs)):
        ref = mcl.Lattice(m, L, sd)
        for n in calls:
            ref.sweep(n[i], b, D)
        assert lat.t == ref.t == sum(n[i] for n in calls)
        assert _digest(lat) == _digest(ref), (m, L, sd)
        ref.free()
        lat.free()


def test_bench_mix_equals_plain_runs(mcl):
    import ctypes

    from paper_2502_18624_amd._lib import GroupTuning
    from paper_2502_18624_amd.autotune import autotune_group
    print("batched bench mix", flush=True)
    saved = GroupTuning()
    mcl.lib().mcl_group_tuning_get(ctypes.byref(saved))
    try:
        specs = _mix(36, 5)
        tune = autotune_group([(m, L) for (m, L, _, _, _) in specs], sweeps_per_call=4, reps=1)
        print("tuning", {k: v for k, v in tune.items() if k != "rows_log2L"}, flush=True)
        _run_mix_against_plain(mcl, specs, 9)
    finally:
        mcl.lib().mcl_group_tuning_set(ctypes.byref(saved))


@pytest.mark.parametrize("wg,split,graph,gsweeps", [(1, 0, 1, 2), (2, 1, 0, 32), (4, 0, 1, 3)])
def test_bench_mix_persistent_grids(mcl, wg, split, graph, gsweeps):
    """The same mix on persistent grids of 1, 2 and 4 workgroups per CU:
    fewer workgroups than tiles, so each eighth of the tile list is claimed
    tile by tile from its counters, which every launch (graph replays
    included) must leave at zero for the next.  The 4096 and 8192 replicas
    take the scalar row walk."""
    import ctypes

    from paper_2502_18624_amd._lib import GroupTuning
    print("batched bench mix, persistent", wg, split, graph, gsweeps, flush=True)
    saved = GroupTuning()
    mcl.lib().mcl_group_tuning_get(ctypes.byref(saved))
    try:
        t = GroupTuning()
        mcl.lib().mcl_group_tuning_get(ctypes.byref(t))
        t.use_graph, t.largest_first, t.wg_per_cu, t.split_models, t.graph_sweeps = graph, 1, wg, split, gsweeps
        assert mcl.lib().mcl_group_tuning_set(ctypes.byref(t)) == 0
        _run_mix_against_plain(mcl, _mix(36, 6 + wg), 10 + wg)
    finally:
        mcl.lib().mcl_group_tuning_set(ctypes.byref(saved))


def test_group_call_with_a_lattice_too_large_to_batch(mcl):
    """A 1-bit lattice of L = 2^17 + 256 (above the batched limit of 2^17)
    beside small replicas: the call sweeps it on its own; light-cone
    windows of the oracle check it."""
    print("group with a large lattice", flush=True)
    L, seed, n = 2**17 + 256, 1201, 3
    big = mcl.Lattice(2, L, seed)
    small = [mcl.Lattice(0, 256, 1202), mcl.Lattice(1, 256, 1203)]
    mcl.group_sweep([big] + small, [n, n, n], [BETA_C] * 3, [0.0, 0.0, 1.0])
    assert big.t == n and all(s.t == n for s in small)
    W, pad = 32, 2 * n
    P = W + 2 * pad
    for (x0, y0) in [(0, 0), (L - 16, L - 16), (L // 2 + 3, 99991 % L)]:
        got = big.read_window(x0, y0, W, W)
        patch = oracle.window_run(2, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, BETA_C)
        assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    for lat, (m, sd, D) in zip(small, [(0, 1202, 0.0), (1, 1203, 1.0)]):
        want = oracle.init(m, 256, sd)
        oracle.sweep(want, m, sd, 0, n, BETA_C, D)
        assert np.array_equal(lat.read(), want)
    big.free()
