"""Parity at the benchmark sizes (Ising L = 2^17, Blume-Capel L = 2^16),
through the same sweep path bench.py times.  The oracle cannot replay a
2^34-site lattice, so it checks light-cone windows: after n sweeps a window
depends only on the initial patch 2n sites wider on every side, which the
oracle's window mode evolves with the global coordinates.  Measurements at
full size are checked through properties that hold at any size, and
through closed forms on ordered states."""
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


def _windows(L):
    return [(0, 0), (L - 24, L - 24), (L // 2 + 7, 12345 % L), (98765 % L, L - 10), (L - 40, 3)]


@pytest.mark.parametrize("model,L,seed,n,beta,D", [
    (0, 2**17, 1002, 6, BETA_C, 0.0),
    (1, 2**16, 1003, 4, 1 / 1.4, 1.0),
])
def test_light_cone_windows_at_full_size(mcl, model, L, seed, n, beta, D):
    print("full-size windows", model, L, flush=True)
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, beta, D)
    W, pad = 48, 2 * n
    P = W + 2 * pad
    for (x0, y0) in _windows(L):
        got = lat.read_window(x0, y0, W, W)
        patch = oracle.window_run(model, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, beta, D)
        assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    lat.free()


def test_measure_invariants_at_full_size(mcl):
    print("full-size measure invariants", flush=True)
    L = 2**17
    lat = mcl.Lattice(mcl.ISING, L, 1002)
    lat.sweep(4, BETA_C)
    m = lat.measure(mcl.CORR_PROTOCOL)
    N = L * L
    assert m["invalid"] == 0 and sum(m["counts"]) == N and m["counts"][1] == 0
    assert m["M"] == m["counts"][2] - m["counts"][0]
    assert m["Q"] == m["counts"][2] + m["counts"][0] == N
    assert m["Cx"][0] == m["Q"] and m["Cy"][0] == m["Q"]
    # Schwinger-Dyson histogram: every site once, sum of sigma h = 2 B, Ising h even
    assert sum(m["sd"]) == N and sum((k - 4) * v for k, v in enumerate(m["sd"])) == 2 * m["B"]
    assert all(v == 0 for v in m["sd"][1::2])
    assert np.array_equal(m["r"], oracle.rset(oracle.CORR_PROTOCOL, L, 4))
    expect_src = np.where(m["r"] <= 32, N, (L // 16) ** 2)
    assert np.array_equal(m["nsrc"], expect_src)
    assert np.all(np.abs(m["Cx"]) <= m["nsrc"]) and np.all(np.abs(m["Cy"]) <= m["nsrc"])
    assert np.all(m["Cx"][1:8] > 0) and np.all(m["Cy"][1:8] > 0)      # short-range order after the quench
    # the same buffer with an ordered state: closed forms at full size
    mem = lat.mem
    lat.free()
    up = mcl.Lattice(mcl.ISING, L, 1, mcl.INIT_UP, mem=mem)
    m = up.measure(mcl.CORR_PROTOCOL)
    assert (m["B"], m["M"], m["Q"]) == (2 * N, N, N)
    assert m["sd"] == [0] * 8 + [N]
    assert np.array_equal(m["Cx"], m["nsrc"]) and np.array_equal(m["Cy"], m["nsrc"])
    up.free()


@pytest.mark.parametrize("model", [0, 1])
def test_protocol_parity_at_4096(mcl, model):
    """Element-by-element parity of every measured sum at L = 4096 (many LDS
    tiles and source rows), after a few sweeps."""
    print("protocol parity 4096", model, flush=True)
    L = 4096
    lat = mcl.Lattice(model, L, 77 + model)
    lat.sweep(3, BETA_C, 1.0)
    s = lat.read()
    want = oracle.init(model, L, 77 + model)
    oracle.sweep(want, model, 77 + model, 0, 3, BETA_C, 1.0, nthreads=8)
    assert np.array_equal(s, want)
    m = lat.measure(mcl.CORR_PROTOCOL)
    om = oracle.measure(s)
    assert (m["B"], m["M"], m["Q"], m["counts"]) == (om["B"], om["M"], om["Q"], om["counts"])
    assert m["sd"] == list(oracle.sd_hist(s))
    Cx, Cy, ns = oracle.corr(s, oracle.CORR_PROTOCOL, m["r"])
    assert np.array_equal(m["Cx"], Cx) and np.array_equal(m["Cy"], Cy) and np.array_equal(m["nsrc"], ns)
