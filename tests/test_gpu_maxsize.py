"""The largest lattices one MI355X holds: Ising with 1-bit cells at L = 2^20
(2^40 spins, 128 GiB, the paper's per-GPU maximum) and with 4-bit cells at
L = 2^19 (128 GiB).  Beyond 2^32 Philox blocks per colour the counter's
high word is nonzero, a path no smaller lattice takes; light-cone windows
of the oracle check it bit for bit, and the full-size measurement is checked
through invariants and closed forms on ordered states."""
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
    free, _ = torch.cuda.mem_get_info()
    if free < 140 * 2**30:
        pytest.skip("needs 140 GiB of free device memory")
    return m


def _release():
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _check_invariants(m, L):
    N = L * L
    assert m["invalid"] == 0 and m["counts"][1] == 0 and m["Q"] == N
    assert m["M"] == m["counts"][2] - m["counts"][0]
    assert m["Cx"][0] == N and m["Cy"][0] == N
    assert sum(m["sd"]) == N and sum((k - 4) * v for k, v in enumerate(m["sd"])) == 2 * m["B"]
    assert all(v == 0 for v in m["sd"][1::2])
    assert np.array_equal(m["nsrc"], np.where(m["r"] <= 32, N, (L // 16) ** 2))
    assert np.all(np.abs(m["Cx"]) <= m["nsrc"]) and np.all(np.abs(m["Cy"]) <= m["nsrc"])
    assert np.all(m["Cx"][1:4] > 0) and np.all(m["Cy"][1:4] > 0)      # short-range order after 2 sweeps


@pytest.mark.parametrize("model,L,seed", [(2, 2**20, 1005), (0, 2**19, 1006)])
def test_largest_lattice(mcl, model, L, seed):
    print("max-size lattice", model, L, flush=True)
    n = 2
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, BETA_C)
    W, pad = 32, 2 * n
    P = W + 2 * pad
    for (x0, y0) in [(0, 0), (L - 16, L - 16), (L // 2 + 5, 777777 % L), (L - 20, 3)]:
        got = lat.read_window(x0, y0, W, W)
        patch = oracle.window_run(model, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, BETA_C)
        assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    m = lat.measure(mcl.CORR_PROTOCOL)
    assert np.array_equal(m["r"], oracle.rset(oracle.CORR_PROTOCOL, L, n))
    _check_invariants(m, L)
    # the same buffer with the all-up state: closed forms at full size
    mem = lat.mem
    lat.free()
    up = mcl.Lattice(model, L, 1, mcl.INIT_UP, mem=mem)
    m = up.measure(mcl.CORR_PROTOCOL)
    N = L * L
    assert (m["B"], m["M"], m["Q"]) == (2 * N, N, N)
    assert m["sd"] == [0] * 8 + [N]
    assert np.array_equal(m["Cx"], m["nsrc"]) and np.array_equal(m["Cy"], m["nsrc"])
    up.free()
    del lat, up, mem
    _release()


@pytest.mark.parametrize("model,L,shift", [(0, 185408, 2), (1, 185408, 2), (2, 370944, 4)])
def test_counter_high_word_changes_inside_a_band(mcl, model, L, shift):
    """L not a power of two, just large enough that the Philox block index
    k >> shift of the in-colour index k passes 2^32 inside the lattice, in
    the middle of a band of rows: the waves there take the per-lane form of
    the counter.  Windows around the crossing against the oracle."""
    print("high word inside a band", model, L, flush=True)
    n, seed, beta, D = 2, 1007, BETA_C if model != 1 else 1 / 1.4, 1.0
    k = 1 << (32 + shift)                           # first in-colour index of block 2^32
    yb, ib = divmod(k, L // 2)
    assert 0 < yb < L - 1
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, beta, D)
    W, pad = 32, 2 * n
    P = W + 2 * pad
    for dx in (-40, 0, 24):
        x0, y0 = (2 * ib + dx) % L, yb - W // 2
        got = lat.read_window(x0, y0, W, W)
        patch = oracle.window_run(model, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, beta, D)
        assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    lat.free()
    del lat
    _release()
