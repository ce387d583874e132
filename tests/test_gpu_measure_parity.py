"""Element-by-element parity of every measured sum with the oracle, on the
launch shapes the benchmark sizes take (section 3.3 protocol; eq. SDI
histogram; B, M, Q and the spin counts).

- L = 32768, all three models, 3 sweeps from the random start: the device
  lattice equals the oracle's, and B, M, Q, counts, sigma-h histogram,
  distances, source counts, C_x and C_y computed by the library equal the
  oracle's sums over that lattice.  At this size every measurement kernel
  runs the branches the 2^17 benchmark runs: workgroups with several tiles
  of the short-distance pass (reusing halo rows), several rows of the
  sampled x pass with several words per lane, several distance chunks of
  the sampled y pass, and the pass that writes the sampled columns' bits
  (for 4-bit Ising cells the short-distance tiles, which give B, M, Q and
  the histogram too; otherwise the B/M/Q pass).  Without correlations
  the B/M/Q pass runs for every model, and gives the same sums.
- The same branches at L <= 4096, forced by capping the grid of the
  measurement kernels (MCL_MEASURE_GRID), in protocol and full mode, with
  several B/M/Q tasks per thread besides, and with the B/M/Q pass's 64-row
  bands of L >= 2^16 (MCL_MEASURE_ROWS); at L = 4096 the 4-bit Ising sums
  both from the short-distance tiles and from the B/M/Q pass
  (MCL_MEASURE_FUSED).
- t = 10^6: r_c(t) exceeds L/2, so every distance up to L/2 is measured and
  each residue class of the sampled distances spans several chunks.
- The L = 256 quench of the parity-size workload in full: seed 1001,
  T = 0.9 T_c, 1000 sweeps, full C(r) along both axes at t = 2^k."""
import math
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


@pytest.fixture(scope="module")
def mcl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_18624_amd as m
    m.lib()
    return m


def _params(model):
    return (1 / 1.4, 1.0) if model == 1 else (BETA_C, 0.0)


def _compare(m, s, mode, nthreads):
    """Every field of measure() against the oracle's sums over s."""
    om = oracle.measure(s, nthreads)
    assert (m["B"], m["M"], m["Q"]) == (om["B"], om["M"], om["Q"])
    assert m["counts"] == om["counts"] and m["invalid"] == 0
    assert m["sd"] == [int(v) for v in oracle.sd_hist(s, nthreads)]
    r = oracle.rset(mode, s.shape[0], m["t"])
    assert np.array_equal(m["r"], r)
    Cx, Cy, ns = oracle.corr(s, mode, r, nthreads)
    assert np.array_equal(m["nsrc"], ns)
    bad_x = np.nonzero(m["Cx"] != Cx)[0]
    bad_y = np.nonzero(m["Cy"] != Cy)[0]
    assert bad_x.size == 0, ("Cx differs at r =", r[bad_x][:10])
    assert bad_y.size == 0, ("Cy differs at r =", r[bad_y][:10])


@pytest.mark.parametrize("model", [0, 1, 2])
def test_measure_parity_at_32768(mcl, model):
    L, seed, n = 32768, 4400 + model, 3
    beta, D = _params(model)
    nt = _threads()
    print("measure parity L=32768 model", model, "threads", nt, flush=True)
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, beta, D)
    m = lat.measure(mcl.CORR_PROTOCOL)
    m0 = lat.measure(mcl.CORR_NONE)
    s = lat.read()
    lat.free()
    for k in ("B", "M", "Q", "counts", "invalid", "sd"):
        assert m0[k] == m[k], k
    want = oracle.init(model, L, seed)
    oracle.sweep(want, model, seed, 0, n, beta, D, nthreads=nt)
    assert np.array_equal(s, want), "lattice differs at %d sites" % int((s != want).sum())
    del want
    _compare(m, s, oracle.CORR_PROTOCOL, nt)


@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("mode,L,grid,rows", [(2, 4096, 3, 0), (2, 4096, 1, 64), (1, 512, 3, 64), (2, 4096, 16, 64)])
def test_measure_parity_split_launches(mcl, monkeypatch, model, mode, L, grid, rows):
    """Three workgroups (or one, or 16) for the persistent passes, so each
    takes several tasks, tiles, sampled rows and groups of source-row
    words, with uneven shares; B/M/Q bands of 64 rows where rows is set."""
    print("measure parity split launches", model, mode, L, grid, rows, flush=True)
    monkeypatch.setenv("MCL_MEASURE_GRID", str(grid))
    if rows:
        monkeypatch.setenv("MCL_MEASURE_ROWS", str(rows))
    beta, D = _params(model)
    lat = mcl.Lattice(model, L, 4500 + model)
    lat.sweep(3, beta, D)
    m = lat.measure(mode)
    s = lat.read()
    want = oracle.init(model, L, 4500 + model)
    oracle.sweep(want, model, 4500 + model, 0, 3, beta, D, nthreads=_threads())
    assert np.array_equal(s, want)
    _compare(m, s, mode, _threads())
    # the knobs change the launch shape only; at L = 4096 the 4-bit Ising
    # sums come from the short-distance tiles, or (MCL_MEASURE_FUSED=0) from
    # the B/M/Q pass
    monkeypatch.delenv("MCL_MEASURE_GRID")
    monkeypatch.delenv("MCL_MEASURE_ROWS", raising=False)
    for fused in ("1", "0"):
        monkeypatch.setenv("MCL_MEASURE_FUSED", fused)
        m2 = lat.measure(mode)
        for k in ("B", "M", "Q", "counts", "sd"):
            assert m2[k] == m[k]
        for k in ("r", "Cx", "Cy", "nsrc"):
            assert np.array_equal(m2[k], m[k])
    monkeypatch.delenv("MCL_MEASURE_FUSED")


@pytest.mark.parametrize("model", [0, 1, 2])
def test_protocol_beyond_half_lattice(mcl, model):
    """t = 10^6 at L = 4096: r_c(t) = floor(g(L) 1000 + 0.5) > L / 2, so the
    linear range runs to L/2 and every residue class of the sampled
    distances holds about 126 of them (four chunks of the y pass)."""
    print("protocol at t=1e6", model, flush=True)
    L, seed, t0, n = 4096, 4600 + model, 10**6, 2
    beta, D = _params(model)
    start = oracle.init(model, L, seed)
    oracle.sweep(start, model, seed, 0, 1, beta, D)
    assert oracle.rc(L, t0 + n) > L // 2
    lat = mcl.Lattice(model, L, seed)
    lat.write(start, t0)
    lat.sweep(n, beta, D)
    m = lat.measure(mcl.CORR_PROTOCOL)
    assert m["t"] == t0 + n
    s = lat.read()
    want = start.copy()
    oracle.sweep(want, model, seed, t0, n, beta, D)
    assert np.array_equal(s, want)
    assert np.array_equal(m["r"], np.arange(L // 2 + 1))
    _compare(m, s, oracle.CORR_PROTOCOL, _threads())


def test_parity_size_quench_in_full(mcl):
    """Ising L = 256, seed 1001, T = 0.9 T_c, random start, 1000 sweeps;
    B, M and the full C(r) along both axes at t = 2^k, k = 0 .. 9, and the
    final lattice, all against the oracle."""
    print("parity-size quench in full", flush=True)
    L, seed, beta, total = 256, 1001, BETA_C / 0.9, 1000
    lat = mcl.Lattice(mcl.ISING, L, seed)
    s = oracle.init(oracle.ISING, L, seed)
    assert np.array_equal(lat.read(), s)
    done = 0
    for t in oracle.schedule_pow2(total) + [total]:
        if t > done:
            lat.sweep(t - done, beta)
            oracle.sweep(s, oracle.ISING, seed, done, t - done, beta)
            done = t
        m = lat.measure(mcl.CORR_FULL)
        assert m["t"] == t
        _compare(m, s, oracle.CORR_FULL, 1)
    assert np.array_equal(lat.read(), s)


@pytest.mark.parametrize("seed", [4700])
def test_fused_tiles_on_a_partial_strip(mcl, monkeypatch, seed):
    """Ising L = 4160 (65 words of a plane row: two strips of 32 words and
    one of a single word), FULL correlations: the short-distance tiles give
    the B/M/Q sums with a partial last strip and no T bits.  B, M, Q, the
    counts and the histogram equal the oracle's, and every sum equals the
    one with the separate B/M/Q pass (MCL_MEASURE_FUSED=0)."""
    print("fused tiles on a partial strip", seed, flush=True)
    L = 4160
    lat = mcl.Lattice(mcl.ISING, L, seed)
    lat.sweep(2, BETA_C)
    m = lat.measure(mcl.CORR_FULL)
    s = lat.read()
    om = oracle.measure(s, _threads())
    assert (m["B"], m["M"], m["Q"]) == (om["B"], om["M"], om["Q"])
    assert m["counts"] == om["counts"] and m["invalid"] == 0
    assert m["sd"] == [int(v) for v in oracle.sd_hist(s, _threads())]
    monkeypatch.setenv("MCL_MEASURE_FUSED", "0")
    m2 = lat.measure(mcl.CORR_FULL)
    for k in ("B", "M", "Q", "counts", "sd"):
        assert m2[k] == m[k], k
    for k in ("r", "Cx", "Cy", "nsrc"):
        assert np.array_equal(m2[k], m[k]), k
    lat.free()


def test_one_bit_measurement_on_a_caller_stream(mcl):
    """1-bit lattices run the sampled y pass on a second stream of the
    handle, forked from and joined back into the lattice's stream.  A lattice
    queued on a stream of the caller's measures the same sums as one on the
    current stream, at sizes where the y pass covers the consecutive and the
    log-spaced distances."""
    import torch
    print("1-bit measurement on a caller stream", flush=True)
    L, seed = 8192, 4800
    side = torch.cuda.Stream()
    a = mcl.Lattice(mcl.ISING_LUT, L, seed, stream=side)
    b = mcl.Lattice(mcl.ISING_LUT, L, seed)
    for lat in (a, b):
        lat.sweep(3, BETA_C)
    ma, mb = a.measure(mcl.CORR_PROTOCOL), b.measure(mcl.CORR_PROTOCOL)
    for k in ("B", "M", "Q", "counts", "sd", "t"):
        assert ma[k] == mb[k], k
    for k in ("r", "Cx", "Cy", "nsrc"):
        assert np.array_equal(ma[k], mb[k]), k
    s = b.read()
    Cx, Cy, _ = oracle.corr(s, oracle.CORR_PROTOCOL, mb["r"], _threads())
    assert np.array_equal(mb["Cy"], Cy) and np.array_equal(mb["Cx"], Cx)
    a.free()
    b.free()
