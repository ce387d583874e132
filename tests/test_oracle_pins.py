"""Pins for the CPU oracle: each test checks the oracle against something
other than itself -- an independent implementation, a closed form, exact
enumeration, an invariant of the dynamics, or values evaluated by hand from
the paper's formulas.  CPU only."""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
TC = 1.0 / BETA_C


# --------------------------------------------------------------------------
# Philox4x32-10: cross-implementation against rocRAND's engine (host code).
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND cross-check")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-o", out, os.path.join(HERE, "pins", "philox_rocrand.cpp")],
                   check=True, cwd="/tmp", capture_output=True)

    def run(rows):
        txt = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
        res = subprocess.run([out], input=txt, capture_output=True, text=True, check=True)
        return [[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()]
    return run


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(12345)
    rows = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 1, 0, 0],
            [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1], [123, 0, 7, 1, 1001, 0]]
    for _ in range(300):
        x = int(rng.integers(0, 2**32))
        y = int(rng.integers(0, 2**30))
        z = int(rng.integers(0, 2**32))
        w = int(rng.integers(0, 2**32))
        k0 = int(rng.integers(0, 2**32))
        k1 = int(rng.integers(0, 2**32))
        rows.append([x, y, z, w, k0, k1])
    ref = rocrand_philox(rows)
    assert len(ref) == len(rows)
    for r, expect in zip(rows, ref):
        assert oracle.philox(r[:4], r[4:]) == expect, r


def test_philox_streams_use_contract_counters(rocrand_philox):
    """The accept / proposal / init streams read the documented counter words."""
    seed = (7 << 32) | 1001
    rows, want = [], []
    for k in [0, 1, 2, 3, 4, 5, 1000, 2**33 + 5, 2**40 + 3]:
        for t, c in [(0, 0), (5, 1), (2**32 - 1, 0)]:
            blk = k >> 2
            rows.append([blk & 0xFFFFFFFF, blk >> 32, t, c, seed & 0xFFFFFFFF, seed >> 32])
            want.append(("acc", k, t, c))
            blk = k >> 7
            rows.append([blk & 0xFFFFFFFF, blk >> 32, t, 2 + c, seed & 0xFFFFFFFF, seed >> 32])
            want.append(("prop", k, t, c))
        blk = k >> 2
        rows.append([blk & 0xFFFFFFFF, blk >> 32, 0, 4, seed & 0xFFFFFFFF, seed >> 32])
        want.append(("init", k, 0, 0))
    ref = rocrand_philox(rows)
    for (kind, k, t, c), out in zip(want, ref):
        if kind == "acc":
            assert oracle.accept_draw(seed, t, c, k) == out[k & 3]
        elif kind == "prop":
            assert oracle.proposal_bit(seed, t, c, k) == (out[(k >> 5) & 3] >> (k & 31)) & 1
        else:
            assert oracle.init_draw(seed, k) == out[k & 3]


def test_philox_bit_balance():
    """Statistical sanity: each output bit is set about half the time."""
    n = 4096
    words = np.array([oracle.philox([i, 0, 3, 1], [99, 0]) for i in range(n)], dtype=np.uint64).ravel()
    bits = np.array([((words >> b) & 1).sum() for b in range(32)], dtype=float)
    m = len(words)
    z = (bits - m / 2) / math.sqrt(m / 4)
    assert np.all(np.abs(z) < 5.0)


# --------------------------------------------------------------------------
# Thresholds: closed forms through Onsager's critical point, and 60-digit
# decimal evaluations of floor(2^32 exp(-beta dE)).
# --------------------------------------------------------------------------
def _dec_threshold(beta_str_or_dec, dE):
    getcontext().prec = 60
    b = Decimal(beta_str_or_dec)
    v = (-(b * Decimal(dE))).exp() * (Decimal(2) ** 32)
    return min(int(v), 2**32 - 1)


def test_thresholds_closed_form_at_beta_c():
    # exp(-2 beta_c) = sqrt(2) - 1 (Onsager), so e^{-4 beta_c} = 3 - 2 sqrt 2
    # and e^{-8 beta_c} = 17 - 12 sqrt 2.
    getcontext().prec = 60
    s2 = Decimal(2).sqrt()
    T4 = int((Decimal(3) - 2 * s2) * Decimal(2) ** 32)
    T8 = int((Decimal(17) - 12 * s2) * Decimal(2) ** 32)
    assert (T4, T8) == (736899888, 126432032)
    assert oracle.ising_thresholds(BETA_C) == (T4, T8)


@pytest.mark.parametrize("frac", [0.5, 0.9, 1.0, 1.5])
def test_thresholds_match_high_precision(frac):
    beta = BETA_C / frac
    bd = Decimal(repr(beta))
    assert oracle.ising_thresholds(beta) == (_dec_threshold(bd, 4), _dec_threshold(bd, 8))


def test_threshold_consistency_identity():
    # e^{-4 beta} at T = Tc/2 equals e^{-8 beta_c}
    assert oracle.ising_thresholds(BETA_C / 0.5)[0] == oracle.ising_thresholds(BETA_C)[1]


def test_threshold_limits():
    assert oracle.threshold(0.0, 4.0) == 2**32 - 1           # beta = 0 clamps
    assert oracle.threshold(float("inf"), 4.0) == 0          # beta = inf never accepts
    assert oracle.threshold(1e-12, 1.0) == 2**32 - 1


def test_bc_table_high_precision():
    beta, D = 1.0 / 1.4, 1.0
    thr, always = oracle.bc_table(beta, D)
    bd = Decimal(repr(beta))
    seen = {}
    for si in range(3):
        for b in range(2):
            for hi in range(9):
                s, h = si - 1, hi - 4
                s2 = ((si + 1 + b) % 3) - 1
                dE = -h * (s2 - s) + D * (s2 * s2 - s * s)
                if dE <= 0:
                    assert always[si, b, hi]
                else:
                    assert not always[si, b, hi]
                    want = _dec_threshold(bd, Decimal(repr(dE)))
                    assert int(thr[si, b, hi]) == want
                    seen[dE] = want
    # positive energy changes reachable at D = 1: 1..6 and 8
    assert sorted(seen) == [1, 2, 3, 4, 5, 6, 8]


# --------------------------------------------------------------------------
# Single-site kernels: exact global balance with the Boltzmann weights of
# eq. (IM) / eq. (BC) for every local field, up to the 2^-32 quantisation.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("beta", [0.1, BETA_C, 0.8, 2.0])
def test_ising_single_site_balance(beta):
    for h in (-4, -2, 0, 2, 4):
        w = {s: math.exp(beta * s * h) for s in (-1, 1)}   # exp(-beta E), E = -s h
        flow = {}
        for s in (-1, 1):
            aligned = (4 + s * h) // 2
            flow[s] = w[s] * oracle.ising_flip_prob(aligned, beta)
        assert abs(flow[1] - flow[-1]) <= 4e-9 * max(w.values())


@pytest.mark.parametrize("beta,D", [(1 / 1.4, 1.0), (0.5, 0.0), (1.0, -0.7), (0.3, 2.5)])
def test_bc_single_site_balance(beta, D):
    for h in range(-4, 5):
        pi = {s: math.exp(-beta * (-s * h + D * s * s)) for s in (-1, 0, 1)}
        P = {}
        for s in (-1, 0, 1):
            stay = 1.0
            for b in (0, 1):
                s2 = ((s + 1 + 1 + b) % 3) - 1
                p = 0.5 * oracle.bc_accept_prob(s, h, b, beta, D)
                P[(s, s2)] = p
                stay -= p
            P[(s, s)] = stay
        for s2 in (-1, 0, 1):
            lhs = sum(pi[s] * P[(s, s2)] for s in (-1, 0, 1))
            assert abs(lhs - pi[s2]) <= 4e-9 * max(pi.values())


# --------------------------------------------------------------------------
# Initial states.
# --------------------------------------------------------------------------
def test_init_random_statistics():
    s = oracle.init(oracle.ISING, 256, 1001)
    N = s.size
    assert set(np.unique(s)) <= {-1, 1}
    assert abs(s.sum()) < 5 * math.sqrt(N)
    b = oracle.init(oracle.BC, 256, 1003)
    for v in (-1, 0, 1):
        c = (b == v).sum()
        assert abs(c - N / 3) < 5 * math.sqrt(N * (1 / 3) * (2 / 3))
    # neighbouring sites are uncorrelated at T = infinity
    for arr in (s, b):
        a = arr.astype(np.int64)
        assert abs((a * np.roll(a, 1, axis=1)).sum()) < 5 * math.sqrt(N)


def test_init_ordered_and_errors():
    assert (oracle.init(oracle.ISING, 8, 0, oracle.INIT_UP) == 1).all()
    assert (oracle.init(oracle.BC, 8, 0, oracle.INIT_DOWN) == -1).all()
    assert (oracle.init(oracle.BC, 8, 0, oracle.INIT_ZERO) == 0).all()
    with pytest.raises(ValueError):
        oracle.init(oracle.ISING, 8, 0, oracle.INIT_ZERO)
    with pytest.raises(ValueError):
        oracle.init(oracle.ISING, 2, 0)


# --------------------------------------------------------------------------
# Exact enumeration vs long oracle runs (within 3 sigma, binned errors).
# --------------------------------------------------------------------------
def _enumerate_ising(L, beta):
    N = L * L
    idx = np.arange(2 ** N, dtype=np.int64)
    spins = (((idx[:, None] >> np.arange(N)) & 1) * 2 - 1).astype(np.int64).reshape(-1, L, L)
    B = (spins * (np.roll(spins, -1, 2) + np.roll(spins, -1, 1))).sum(axis=(1, 2))
    M = spins.sum(axis=(1, 2))
    E = -B
    w = np.exp(-beta * (E - E.min()))
    Z = w.sum()
    return {"E": (w * E).sum() / Z, "M2": (w * M * M).sum() / Z, "absM": (w * np.abs(M)).sum() / Z}


def _enumerate_bc(L, beta, D):
    """Exact averages over all 3^(L*L) states, in chunks of 3^(N-4) states."""
    N = L * L
    rest = N - 4 if N > 4 else N
    idx = np.arange(3 ** rest, dtype=np.int64)
    low = np.empty((3 ** rest, rest), dtype=np.int8)
    rem = idx.copy()
    for j in range(rest):
        low[:, j] = rem % 3
        rem //= 3
    low -= 1
    acc = {"Z": 0.0, "E": 0.0, "M2": 0.0, "absM": 0.0, "Q": 0.0}
    shift = None
    for head in range(3 ** (N - rest)):
        hd = np.array([(head // 3 ** j) % 3 - 1 for j in range(N - rest)], dtype=np.int8)
        spins = np.concatenate([np.broadcast_to(hd, (len(low), N - rest)), low], axis=1)
        spins = spins.reshape(-1, L, L).astype(np.int32)
        B = (spins * (np.roll(spins, -1, 2) + np.roll(spins, -1, 1))).sum(axis=(1, 2))
        M = spins.sum(axis=(1, 2)).astype(np.float64)
        Q = (spins * spins).sum(axis=(1, 2))
        E = -B + D * Q
        if shift is None:
            shift = -2.0 * N - abs(D) * N     # lower bound of E, keeps weights finite
        w = np.exp(-beta * (E - shift))
        acc["Z"] += w.sum()
        acc["E"] += (w * E).sum()
        acc["M2"] += (w * M * M).sum()
        acc["absM"] += (w * np.abs(M)).sum()
        acc["Q"] += (w * Q).sum()
    Z = acc.pop("Z")
    return {k: v / Z for k, v in acc.items()}


def _binned(x, nbins=100):
    x = np.asarray(x, dtype=float)
    n = len(x) // nbins * nbins
    means = x[:n].reshape(nbins, -1).mean(axis=1)
    return means.mean(), means.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.parametrize("beta", [0.3, BETA_C, 0.6])
def test_ising_4x4_enumeration(beta):
    L = 4
    exact = _enumerate_ising(L, beta)
    s = oracle.init(oracle.ISING, L, 77)
    oracle.sweep(s, oracle.ISING, 77, 0, 200, beta)
    Bs, Ms, _ = oracle.series(s, oracle.ISING, 77, 200, 200000, beta)
    for key, series in (("E", -Bs), ("M2", Ms.astype(float) ** 2), ("absM", np.abs(Ms))):
        m, err = _binned(series)
        assert abs(m - exact[key]) < 3 * err + 1e-12, (key, m, exact[key], err)


@pytest.mark.parametrize("beta,D", [(1 / 1.4, 1.0), (0.5, 0.0), (0.9, -0.5)])
def test_bc_3x3_enumeration(beta, D):
    L = 3
    exact = _enumerate_bc(L, beta, D)
    s = oracle.init(oracle.BC, L, 5)
    oracle.sweep(s, oracle.BC, 5, 0, 200, beta, D)
    Bs, Ms, Qs = oracle.series(s, oracle.BC, 5, 200, 200000, beta, D)
    E = -Bs + D * Qs
    for key, series in (("E", E), ("M2", Ms.astype(float) ** 2), ("absM", np.abs(Ms)), ("Q", Qs)):
        m, err = _binned(series)
        assert abs(m - exact[key]) < 3 * err + 1e-12, (key, m, exact[key], err)


def test_bc_4x4_enumeration_energy():
    """Even L: the colour-parallel chain of the GPU path, 3^16 states."""
    L, beta, D = 4, 1 / 1.4, 1.0
    exact = _enumerate_bc(L, beta, D)
    s = oracle.init(oracle.BC, L, 9)
    oracle.sweep(s, oracle.BC, 9, 0, 200, beta, D)
    Bs, Ms, Qs = oracle.series(s, oracle.BC, 9, 200, 200000, beta, D)
    for key, series in (("E", -Bs + D * Qs), ("Q", Qs), ("M2", Ms.astype(float) ** 2)):
        m, err = _binned(series)
        assert abs(m - exact[key]) < 3 * err, (key, m, exact[key], err)


# --------------------------------------------------------------------------
# Invariants of the dynamics.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model,L,D", [(oracle.ISING, 16, 0.0), (oracle.BC, 16, 0.7),
                                       (oracle.ISING, 7, 0.0), (oracle.BC, 9, -1.0)])
def test_delta_e_bookkeeping(model, L, D):
    """B and Q after n sweeps equal the start plus the accepted changes."""
    s = oracle.init(model, L, 31)
    m0 = oracle.measure(s)
    dB, dQ = oracle.sweep(s, model, 31, 0, 25, 0.45, D, track=True)
    m1 = oracle.measure(s)
    assert m1["B"] == m0["B"] + dB
    assert m1["Q"] == m0["Q"] + dQ
    assert dB != 0


@pytest.mark.parametrize("model,D", [(oracle.ISING, 0.0), (oracle.BC, 0.0), (oracle.BC, 1.0),
                                     (oracle.BC, -1.5)])
def test_zero_temperature_is_monotone(model, D):
    s = oracle.init(model, 32, 4)
    m = oracle.measure(s)
    e_prev = -m["B"] + D * m["Q"]
    for t in range(30):
        oracle.sweep(s, model, 4, t, 1, float("inf"), D)
        m = oracle.measure(s)
        e = -m["B"] + D * m["Q"]
        assert e <= e_prev
        e_prev = e


def _aligned(s, x, y):
    L = s.shape[0]
    v = s[y, x]
    return sum(int(n == v) for n in (s[y, (x + 1) % L], s[y, (x - 1) % L], s[(y + 1) % L, x], s[(y - 1) % L, x]))


@pytest.mark.parametrize("model", [oracle.ISING, oracle.ISING_LUT])
def test_zero_temperature_limit_is_the_majority_rule(model):
    """At beta = infinity the Metropolis rule of section 3.2 needs no random
    numbers: e^{-4 beta} = e^{-8 beta} = 0, so a spin flips iff dE <= 0, i.e.
    iff at most two of its four neighbours are aligned (ties flip).  One sweep
    equals that deterministic rule applied to colour 0, then to colour 1."""
    for seed in (1, 2, 3):
        L = 10
        s = oracle.init(model, L, seed)
        ref = s.copy()
        oracle.sweep(s, model, seed, 0, 1, float("inf"))
        for c in (0, 1):
            flips = [(x, y) for y in range(L) for x in range(L) if (x + y) % 2 == c and _aligned(ref, x, y) <= 2]
            for x, y in flips:
                ref[y, x] = -ref[y, x]
        assert np.array_equal(s, ref), (model, seed)


@pytest.mark.parametrize("model", [oracle.ISING, oracle.ISING_LUT])
def test_infinite_temperature_flips_every_spin(model):
    """At beta = 0 every Ising move is accepted (4-bit: u < 2^32 - 1, which
    these seeds never miss; 1-bit: p = 1 sets every pattern bit), so each
    sweep maps s to -s."""
    s = oracle.init(model, 16, 9)
    s0 = s.copy()
    oracle.sweep(s, model, 9, 0, 1, 0.0)
    assert np.array_equal(s, -s0)
    oracle.sweep(s, model, 9, 1, 1, 0.0)
    assert np.array_equal(s, s0)


def test_sweep_uses_the_contract_draws():
    """The counter plumbing of a sweep: after sweep t from s0, every colour-0
    site (updated first, from colour-1 neighbours still as in s0) has flipped
    exactly as the section 3.2 rule says for its accept draw u(seed, t, 0, k),
    k = (y L + x) >> 1 -- the draw whose values the rocRAND pin fixes.  At
    e^{-4 beta} = 1/2 about half the draw-dependent sites flip."""
    beta = math.log(2.0) / 4.0
    T4, T8 = oracle.ising_thresholds(beta)
    L, seed, checked = 16, 77, 0
    for t in (0, 5, 123456):
        s0 = oracle.init(oracle.ISING, L, seed + t)
        s = s0.copy()
        oracle.sweep(s, oracle.ISING, seed, t, 1, beta)
        for y in range(L):
            for x in range(L):
                if (x + y) % 2:
                    continue
                a = _aligned(s0, x, y)
                if a <= 2:
                    want = True
                else:
                    u = oracle.accept_draw(seed, t, 0, (y * L + x) >> 1)
                    want = u < (T4 if a == 3 else T8)
                    checked += 1
                assert (s[y, x] == -s0[y, x]) == want, (t, x, y)
    assert checked > 50


def test_ising_global_flip_symmetry():
    """Acceptance depends only on the aligned count, so the trajectory from
    -s0 is exactly minus the trajectory from s0."""
    s = oracle.init(oracle.ISING, 32, 11)
    r = (-s).astype(np.int8)
    for t in range(20):
        oracle.sweep(s, oracle.ISING, 11, t, 1, BETA_C)
        oracle.sweep(r, oracle.ISING, 11, t, 1, BETA_C)
        assert np.array_equal(r, -s)


def test_colour_order_and_sweep_splitting():
    """n sweeps in one call equal n single-sweep calls; threads do not change
    the result for even L."""
    for model, D in ((oracle.ISING, 0.0), (oracle.BC, 0.5)):
        a = oracle.init(model, 24, 3)
        b = a.copy()
        c = a.copy()
        oracle.sweep(a, model, 3, 10, 6, 0.5, D)
        for t in range(10, 16):
            oracle.sweep(b, model, 3, t, 1, 0.5, D)
        oracle.sweep(c, model, 3, 10, 6, 0.5, D, nthreads=4)
        assert np.array_equal(a, b) and np.array_equal(a, c)


# --------------------------------------------------------------------------
# Equilibrium physics: Onsager's energy and Yang's magnetisation, and the
# Schwinger-Dyson identity (eq. SDI).
# --------------------------------------------------------------------------
def _onsager_energy(beta):
    from scipy.special import ellipk
    k = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = ellipk(k * k)
    return -1 / math.tanh(2 * beta) * (1 + 2 / math.pi * (2 * math.tanh(2 * beta) ** 2 - 1) * K)


def test_onsager_yang_at_0p9_tc():
    beta = BETA_C / 0.9
    L = 64
    s = oracle.init(oracle.ISING, L, 2, oracle.INIT_UP)
    oracle.sweep(s, oracle.ISING, 2, 0, 300, beta)
    Bs, Ms, _ = oracle.series(s, oracle.ISING, 2, 300, 4000, beta)
    N = L * L
    e, de = _binned(-Bs / N, 40)
    m, dm = _binned(np.abs(Ms) / N, 40)
    m_yang = (1 - math.sinh(2 * beta) ** -4) ** 0.125
    # finite-size corrections at L = 64 are exponentially small below T_c
    assert abs(e - _onsager_energy(beta)) < 3 * de + 2e-3, (e, _onsager_energy(beta), de)
    assert abs(m - m_yang) < 3 * dm + 2e-3, (m, m_yang, dm)


@pytest.mark.parametrize("model,beta,D,init", [
    (oracle.ISING, 0.3, 0.0, oracle.INIT_RANDOM),      # T > T_c
    (oracle.ISING, 0.6, 0.0, oracle.INIT_UP),          # ordered phase
    (oracle.BC, 0.5, 0.5, oracle.INIT_RANDOM),         # paramagnetic
    (oracle.BC, 1.0, 0.0, oracle.INIT_UP)])            # ordered
def test_schwinger_dyson_identity(model, beta, D, init):
    """Equilibrium holds the identity exactly; off criticality the chain
    equilibrates in a few sweeps, so the binned error is honest."""
    L = 16
    s = oracle.init(model, L, 8, init)
    oracle.sweep(s, model, 8, 0, 300, beta, D)
    vals = []
    for t in range(300, 6300):
        oracle.sweep(s, model, 8, t, 1, beta, D)
        h = oracle.sd_hist(s)
        vals.append(sum(h[k] * math.exp(-2 * beta * (k - 4)) for k in range(9)) / (L * L))
    m, err = _binned(vals, 30)
    assert abs(m - 1.0) < 3 * err, (m, err)


def test_sd_hist_values():
    s = oracle.init(oracle.ISING, 16, 1, oracle.INIT_UP)
    h = oracle.sd_hist(s)
    assert h[8] == 256 and h.sum() == 256
    b = oracle.init(oracle.BC, 16, 1, oracle.INIT_ZERO)
    assert oracle.sd_hist(b)[4] == 256


# --------------------------------------------------------------------------
# Measurements: closed forms on structured states.
# --------------------------------------------------------------------------
def _structured(L, kind):
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    if kind == "up":
        return np.ones((L, L), dtype=np.int8)
    if kind == "checker":
        return np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    if kind == "stripes":
        return np.where(np.broadcast_to(x % 2 == 0, (L, L)), 1, -1).astype(np.int8)
    raise ValueError(kind)


def test_measure_closed_forms():
    L = 16
    N = L * L
    m = oracle.measure(_structured(L, "up"))
    assert (m["B"], m["M"], m["Q"], m["counts"]) == (2 * N, N, N, [0, 0, N])
    m = oracle.measure(_structured(L, "checker"))
    assert (m["B"], m["M"], m["Q"]) == (-2 * N, 0, N)
    m = oracle.measure(_structured(L, "stripes"))
    assert (m["B"], m["M"]) == (0, 0)     # x bonds all -1, y bonds all +1
    b = oracle.init(oracle.BC, L, 0, oracle.INIT_ZERO)
    m = oracle.measure(b)
    assert (m["B"], m["M"], m["Q"], m["counts"]) == (0, 0, 0, [0, N, 0])


@pytest.mark.parametrize("mode", [oracle.CORR_FULL, oracle.CORR_PROTOCOL])
def test_corr_closed_forms(mode):
    L = 128
    r = oracle.rset(mode, L, 4)
    full = L * L
    sampled = (L // 16) ** 2
    cnt = np.array([full if (mode == oracle.CORR_FULL or d <= 32) else sampled for d in r])
    sign = np.where(r % 2 == 0, 1, -1)
    Cx, Cy, ns = oracle.corr(_structured(L, "up"), mode, r)
    assert np.array_equal(ns, cnt) and np.array_equal(Cx, cnt) and np.array_equal(Cy, cnt)
    Cx, Cy, ns = oracle.corr(_structured(L, "checker"), mode, r)
    assert np.array_equal(Cx, sign * cnt) and np.array_equal(Cy, sign * cnt)
    Cx, Cy, ns = oracle.corr(_structured(L, "stripes"), mode, r)
    assert np.array_equal(Cx, sign * cnt) and np.array_equal(Cy, cnt)


def test_corr_zero_distance_and_periodicity():
    L = 32
    b = oracle.init(oracle.BC, L, 17)
    Q = oracle.measure(b)["Q"]
    r = np.arange(L, dtype=np.int32)
    Cx, Cy, ns = oracle.corr(b, oracle.CORR_FULL, r)
    assert Cx[0] == Q and Cy[0] == Q
    for d in range(1, L):
        assert Cx[d] == Cx[L - d] and Cy[d] == Cy[L - d]


def test_corr_random_state_is_uncorrelated():
    L = 128
    s = oracle.init(oracle.ISING, L, 5)
    r = np.array([1, 2, 3, 7, 16, 33, 64], dtype=np.int32)
    Cx, Cy, ns = oracle.corr(s, oracle.CORR_PROTOCOL, r)
    assert np.all(np.abs(Cx) < 5 * np.sqrt(ns)) and np.all(np.abs(Cy) < 5 * np.sqrt(ns))


# --------------------------------------------------------------------------
# Protocol distances and the measurement schedule (hand-evaluated values).
# --------------------------------------------------------------------------
def _golden(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("=")
            out[tuple(lhs.split())] = rhs.split()
    return out


def test_rset_worked_values():
    gold = _golden("rset_protocol.txt")
    for key, val in gold.items():
        kind, args = key[0], [int(a) for a in key[1:]]
        if kind == "g":
            assert abs(oracle.g(args[0]) - float(val[0])) < 5e-5
        elif kind == "rc":
            assert oracle.rc(*args) == int(val[0])
        else:
            L, t = args
            r = oracle.rset(oracle.CORR_PROTOCOL, L, t)
            logp = r[r > oracle.rc(L, t)]
            if kind == "count":
                assert len(r) == int(val[0])
            elif kind == "log_count":
                assert len(logp) == int(val[0])
            elif kind == "log_first3":
                assert list(logp[:3]) == [int(v) for v in val]
            elif kind == "log_last3":
                assert list(logp[-3:]) == [int(v) for v in val]
            elif kind == "log_first":
                assert logp[0] == int(val[0])
            elif kind == "log_last":
                assert logp[-1] == int(val[0])
            else:
                raise AssertionError(kind)


def test_rset_structure():
    for L in (64, 256, 1024, 2**17):
        for t in (1, 100, 2000, 10**6):
            r = oracle.rset(oracle.CORR_PROTOCOL, L, t)
            assert np.all(np.diff(r) > 0) and r[0] == 0 and r[-1] == min(L // 2, r[-1])
            assert r[-1] == L // 2
            assert list(r[:min(33, L // 2 + 1)]) == list(range(min(33, L // 2 + 1)))
    r = oracle.rset(oracle.CORR_FULL, 256)
    assert list(r) == list(range(129))


def test_schedule_worked_values():
    gold = _golden("schedule.txt")
    assert oracle.schedule_paper(1000)[:17] == [int(v) for v in gold[("first",)]]
    assert len(oracle.schedule_paper(1000)) == int(gold[("distinct_upto", "1000")][0])
    assert len(oracle.schedule_paper(2000)) == int(gold[("distinct_upto", "2000")][0])
    assert oracle.schedule_pow2(1000) == [2**k for k in range(10)]
    assert oracle.schedule_pow2(2000) == [2**k for k in range(11)]
    assert set(oracle.schedule_pow2(2000)) <= set(oracle.schedule_paper(2000))


# --------------------------------------------------------------------------
# Light-cone windows: the window mode equals the full-lattice oracle on the
# sites at least 2n from the patch edge (and differs near the edge, which
# shows the frozen ring matters).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model,D", [(oracle.ISING, 0.0), (oracle.BC, 1.0)])
def test_light_cone_window_matches_full_lattice(model, D):
    L, seed, n, P = 64, 1234, 5, 40
    full = oracle.init(model, L, seed)
    oracle.sweep(full, model, seed, 0, n, 0.5, D)
    inner = 2 * n
    for (x0, y0) in [(0, 0), (50, 3), (40, 45), (13, 60)]:
        win = oracle.window_run(model, L, seed, x0, y0, P, n, 0.5, D)
        ys = (y0 + np.arange(P)) % L
        xs = (x0 + np.arange(P)) % L
        ref = full[np.ix_(ys, xs)]
        assert np.array_equal(win[inner:P - inner, inner:P - inner], ref[inner:P - inner, inner:P - inner])
        assert not np.array_equal(win, ref)


# --------------------------------------------------------------------------
# Table-driven random bits (section 3.2) for the 1-bit Ising mode.
# --------------------------------------------------------------------------
def _exact_table(beta):
    from fractions import Fraction
    p = Fraction(math.exp(-4.0 * beta))          # the same double p, then exact arithmetic
    T, cum = [], Fraction(0)
    for k in range(16):
        T.append(math.floor(cum * 2**32))
        prob = Fraction(1)
        for j in range(4):
            prob *= p if (k >> j) & 1 else (1 - p)
        cum += prob
    return T, float(p)


@pytest.mark.parametrize("beta", [0.1, BETA_C, BETA_C / 0.9, 1.0, 3.0])
def test_lut_table_against_exact_rationals(beta):
    T = oracle.lut_table(beta)
    exact, p = _exact_table(beta)
    assert T[0] == 0 and all(a <= b for a, b in zip(T, T[1:]))
    assert all(abs(a - b) <= 1 for a, b in zip(T, exact))
    # each pattern bit is Bernoulli(p) and pairs are independent, to the 2^-32 grid
    w = [((T[k + 1] if k < 15 else 2**32) - T[k]) / 2**32 for k in range(16)]
    for j in range(4):
        assert abs(sum(w[k] for k in range(16) if (k >> j) & 1) - p) < 20 * 2**-32
        for i in range(j):
            both = sum(w[k] for k in range(16) if (k >> j) & 1 and (k >> i) & 1)
            assert abs(both - p * p) < 20 * 2**-32


def test_lut_limits_and_lookup():
    import bisect
    T = oracle.lut_table(float("inf"))           # p = 0: only pattern 0
    assert T[0] == 0 and all(v == 2**32 for v in T[1:])
    assert oracle.lut_lookup(T, 2**32 - 1) == 0
    T = oracle.lut_table(0.0)                    # p = 1: only pattern 15
    assert all(v == 0 for v in T)
    assert oracle.lut_lookup(T, 0) == 15
    T = oracle.lut_table(BETA_C)
    rng = np.random.default_rng(1)
    for u in list(rng.integers(0, 2**32, 2000)) + T[1:] + [t - 1 for t in T[1:]] + [0, 2**32 - 1]:
        assert oracle.lut_lookup(T, int(u)) == bisect.bisect_right(T, int(u)) - 1


def test_lut_draws_use_contract_counters(rocrand_philox):
    seed = 987654321123
    rows, want = [], []
    for g in [0, 1, 5, 77, 2**33 + 3]:
        for t, c, e in [(0, 0, 0), (3, 1, 1), (9, 0, 1)]:
            b = g >> 2
            rows.append([b & 0xFFFFFFFF, b >> 32, t, 8 + 2 * c + e, seed & 0xFFFFFFFF, seed >> 32])
            want.append((g, t, c, e))
    for (g, t, c, e), out in zip(want, rocrand_philox(rows)):
        assert oracle.lut_draw(seed, t, c, e, g) == out[g & 3]


@pytest.mark.parametrize("beta", [0.2, BETA_C, 0.7])
def test_lut_rule_single_site_balance(beta):
    """Flip probabilities implied by the table: e^{-4 beta} with three aligned
    neighbours (one stream), e^{-8 beta} with four (both streams)."""
    T = oracle.lut_table(beta)
    w = [((T[k + 1] if k < 15 else 2**32) - T[k]) / 2**32 for k in range(16)]
    for j in range(4):
        p1 = sum(w[k] for k in range(16) if (k >> j) & 1)
        for h in (2, 4):                      # s h = 2: three aligned; 4: four aligned
            prob = p1 if h == 2 else p1 * p1
            assert abs(math.exp(beta * h) * prob - math.exp(-beta * h)) < 1e-7 * math.exp(beta * h)


@pytest.mark.parametrize("beta", [0.3, BETA_C, 0.6])
def test_lut_ising_4x4_enumeration(beta):
    L = 4
    exact = _enumerate_ising(L, beta)
    s = oracle.init(oracle.ISING_LUT, L, 55)
    oracle.sweep(s, oracle.ISING_LUT, 55, 0, 200, beta)
    Bs, Ms, _ = oracle.series(s, oracle.ISING_LUT, 55, 200, 200000, beta)
    for key, series in (("E", -Bs), ("M2", Ms.astype(float) ** 2), ("absM", np.abs(Ms))):
        m, err = _binned(series)
        assert abs(m - exact[key]) < 3 * err + 1e-12, (key, m, exact[key], err)


def test_lut_ising_invariants():
    s = oracle.init(oracle.ISING_LUT, 32, 4)
    m = oracle.measure(s)
    b_prev = m["B"]
    for t in range(20):                       # beta = infinity: B never decreases
        oracle.sweep(s, oracle.ISING_LUT, 4, t, 1, float("inf"))
        b = oracle.measure(s)["B"]
        assert b >= b_prev
        b_prev = b
    a = oracle.init(oracle.ISING_LUT, 32, 6)
    r = (-a).astype(np.int8)
    for t in range(15):                       # global flip symmetry
        oracle.sweep(a, oracle.ISING_LUT, 6, t, 1, BETA_C)
        oracle.sweep(r, oracle.ISING_LUT, 6, t, 1, BETA_C)
        assert np.array_equal(r, -a)
    c = oracle.init(oracle.ISING_LUT, 16, 3)
    m0 = oracle.measure(c)
    dB, _ = oracle.sweep(c, oracle.ISING_LUT, 3, 0, 10, 0.45, track=True)
    assert oracle.measure(c)["B"] == m0["B"] + dB


def test_lut_window_matches_full_lattice():
    L, seed, n, P = 64, 99, 4, 36
    full = oracle.init(oracle.ISING_LUT, L, seed)
    oracle.sweep(full, oracle.ISING_LUT, seed, 0, n, BETA_C)
    win = oracle.window_run(oracle.ISING_LUT, L, seed, 30, 50, P, n, BETA_C)
    ref = full[np.ix_((50 + np.arange(P)) % L, (30 + np.arange(P)) % L)]
    assert np.array_equal(win[2 * n:P - 2 * n, 2 * n:P - 2 * n], ref[2 * n:P - 2 * n, 2 * n:P - 2 * n])
