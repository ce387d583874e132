"""GPU vs oracle for the 1-bit Ising mode (one bit per spin, random bits
drawn through the 16-entry table of section 3.2), bit-exact: lattices after
n sweeps, checkpoints, the batched path, every measured sum, and light-cone
windows at L = 2^17.  Sizes span one 16-byte vector per row (L = 256) to
many, including L not a power of two."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2
INF = float("inf")
LUT = 2


@pytest.fixture(scope="module")
def mcl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_18624_amd as m
    m.lib()
    return m


def _oracle_run(L, seed, init, n, beta, t0=0, start=None):
    s = oracle.init(LUT, L, seed, init) if start is None else start.copy()
    if n:
        oracle.sweep(s, LUT, seed, t0, n, beta, 0.0, nthreads=8 if L >= 2048 else 1)
    return s


@pytest.mark.parametrize("init", [0, 1, 2])
@pytest.mark.parametrize("L", [256, 768, 1024])
def test_init_parity(mcl, init, L):
    print("lut init parity", init, L, flush=True)
    lat = mcl.Lattice(LUT, L, 2001 + L, init)
    assert np.array_equal(lat.read(), oracle.init(LUT, L, 2001 + L, init))


CASES = [
    (256, 1, 1, BETA_C / 0.9), (256, 2, 17, BETA_C), (512, 3, 3, BETA_C / 0.5), (768, 4, 5, BETA_C / 1.5),
    (256, 5, 2, INF), (1024, 6, 4, BETA_C), (512, 7, 3, 0.0), (2048, 8, 2, BETA_C / 0.9), (256, 9, 9, 3.0),
    (512, 10, 6, 0.8), (256, 12, 4, 1.2),
]


@pytest.mark.parametrize("L,seed,n,beta", CASES)
def test_sweep_parity(mcl, L, seed, n, beta):
    print("lut sweep parity", L, seed, n, beta, flush=True)
    lat = mcl.Lattice(LUT, L, seed)
    lat.sweep(n, beta)
    got = lat.read()
    want = _oracle_run(L, seed, 0, n, beta)
    assert lat.t == n
    assert np.array_equal(got, want), "mismatch at %d cells" % int((got != want).sum())


def test_sweep_parity_over_beta(mcl):
    """Many temperatures, including those where several thresholds of the
    table fall within 2^-12 of each other (low T) and the lookup takes its
    exact search, and beta where p^4 straddles 2^-12."""
    L = 256
    for i, beta in enumerate([0.05, 0.2, 0.35, BETA_C, 0.5, 0.52, 0.53, 0.6, 0.7, 1.0, 1.5, 2.0, 4.0, 8.0]):
        lat = mcl.Lattice(LUT, L, 300 + i)
        lat.sweep(3, beta)
        assert np.array_equal(lat.read(), _oracle_run(L, 300 + i, 0, 3, beta)), beta
        lat.free()


@pytest.mark.parametrize("model,beta", [(LUT, INF), (LUT, 0.0), (0, INF)])
def test_update_rule_truth_table(mcl, model, beta):
    """Deterministic limits of the Ising rule (eq. IM; random bits of section
    3.2 in the 1-bit mode).  At beta = infinity no random bit is set and a
    spin flips iff at most 2 of its 4 neighbours are aligned; at beta = 0
    (1-bit mode) every bit is set and every spin flips.  One sweep from a
    random state in which all 32 (spin, neighbours) cases occur, against the
    colour-by-colour rule written out in numpy."""
    L = 256
    s0 = np.random.default_rng(8).choice([-1, 1], size=(L, L)).astype(np.int8)

    def nsum(a):
        return np.roll(a, 1, 0) + np.roll(a, -1, 0) + np.roll(a, 1, 1) + np.roll(a, -1, 1)

    yy, xx = np.indices((L, L))
    bits = [(s0 > 0)] + [np.roll(s0, sh, ax) > 0 for sh, ax in ((1, 0), (-1, 0), (1, 1), (-1, 1))]
    code = sum(b.astype(np.int64) << j for j, b in enumerate(bits))
    assert len(np.unique(code[((xx + yy) & 1) == 0])) == 32
    want = s0.astype(np.int64)
    for c in (0, 1):
        colour = ((xx + yy) & 1) == c
        flip = colour & ((want * nsum(want) <= 0) if beta == INF else True)   # s h <= 0: at most 2 aligned
        want = np.where(flip, -want, want)
    lat = mcl.Lattice(model, L, 5)
    lat.write(s0, 0)
    lat.sweep(1, beta)
    assert np.array_equal(lat.read(), want.astype(np.int8))


def test_ordered_start_at_zero_temperature_stays(mcl):
    """beta = infinity from the all-up state: every site is aligned with all
    its neighbours, p = 0, so no move is ever accepted."""
    lat = mcl.Lattice(LUT, 512, 3, mcl.INIT_UP)
    lat.sweep(5, INF)
    assert np.all(lat.read() == 1)


def test_split_calls_restart_and_packed(mcl):
    print("lut split/restart", flush=True)
    L, seed, beta = 256, 77, BETA_C / 0.9
    a = mcl.Lattice(LUT, L, seed)
    for n in (3, 1, 13):
        a.sweep(n, beta)
    assert np.array_equal(a.read(), _oracle_run(L, seed, 0, 17, beta))
    snap, t = a.read(), a.t
    b = mcl.Lattice(LUT, L, seed)
    b.write(snap, t)
    b.sweep(5, beta)
    a.sweep(5, beta)
    assert np.array_equal(a.read(), b.read())
    assert np.array_equal(b.read(), _oracle_run(L, seed, 0, 5, beta, t0=17, start=snap))
    packed = a.read_packed()
    assert packed.nbytes == L * L // 8
    c = mcl.Lattice(LUT, L, seed)
    c.write_packed(packed, a.t)
    c.sweep(2, beta)
    a.sweep(2, beta)
    assert np.array_equal(a.read(), c.read())


def test_write_rejects_zero_spins(mcl):
    lat = mcl.Lattice(LUT, 256, 1)
    with pytest.raises(mcl.MclError):
        lat.write(np.zeros((256, 256), dtype=np.int8), 0)


def _check_measure(mcl, lat, mode):
    s = lat.read()
    m = lat.measure(mode)
    om = oracle.measure(s)
    assert (m["B"], m["M"], m["Q"], m["counts"], m["invalid"]) == (om["B"], om["M"], om["Q"], om["counts"], 0)
    assert m["sd"] == list(oracle.sd_hist(s))
    if mode != mcl.CORR_NONE:
        r = oracle.rset(mode, lat.L, lat.t)
        assert np.array_equal(m["r"], r)
        Cx, Cy, ns = oracle.corr(s, mode, r)
        assert np.array_equal(m["nsrc"], ns)
        assert np.array_equal(m["Cx"], Cx), np.nonzero(m["Cx"] != Cx)
        assert np.array_equal(m["Cy"], Cy), np.nonzero(m["Cy"] != Cy)


@pytest.mark.parametrize("L,n", [(256, 3), (512, 8), (768, 2)])
def test_measure_full_parity(mcl, L, n):
    print("lut measure full", L, n, flush=True)
    lat = mcl.Lattice(LUT, L, 4242)
    lat.sweep(n, BETA_C / 0.9)
    _check_measure(mcl, lat, mcl.CORR_FULL)


@pytest.mark.parametrize("L,n", [(256, 1), (1024, 16), (4096, 3)])
def test_measure_protocol_parity(mcl, L, n):
    print("lut measure protocol", L, n, flush=True)
    lat = mcl.Lattice(LUT, L, 99)
    lat.sweep(n, BETA_C)
    _check_measure(mcl, lat, mcl.CORR_PROTOCOL)
    _check_measure(mcl, lat, mcl.CORR_NONE)


def test_measure_ordered_states(mcl):
    L = 1024
    N = L * L
    for init, val in ((1, 1), (2, -1)):
        m = mcl.Lattice(LUT, L, 0, init).measure(mcl.CORR_PROTOCOL)
        assert (m["B"], m["M"], m["Q"]) == (2 * N, val * N, N)
        assert m["sd"] == [0] * 8 + [N]
        assert np.array_equal(m["Cx"], m["nsrc"]) and np.array_equal(m["Cy"], m["nsrc"])


def test_group_sweep_with_one_bit_replicas(mcl):
    """Mixed groups: 1-bit replicas (each with its own bucket table, built by
    the call) advance in the same batched launches as the 4-bit ones; all
    equal the oracle, including a 1-bit temperature whose table needs the
    exact search."""
    rng = np.random.default_rng(11)
    specs = []
    for i in range(6):
        model = (0, 1, LUT)[i % 3]
        L = int(rng.choice([256, 512]))
        specs.append((model, L, 5000 + i, int(rng.integers(1, 5)), float(rng.uniform(0.5, 1.5)) * BETA_C,
                      float(rng.choice([0.0, 1.0]))))
    specs.append((LUT, 256, 5100, 3, 2.0, 0.0))             # many buckets hold several thresholds
    specs.append((LUT, 512, 5101, 2, float("inf"), 0.0))
    lats = [mcl.Lattice(m, L, s) for (m, L, s, _, _, _) in specs]
    mcl.group_sweep(lats, [sp[3] for sp in specs], [sp[4] for sp in specs], [sp[5] for sp in specs])
    for lat, (m, L, s, n, b, D) in zip(lats, specs):
        assert lat.t == n
        want = oracle.init(m, L, s)
        oracle.sweep(want, m, s, 0, n, b, D)
        assert np.array_equal(lat.read(), want), (m, L, n)


def test_light_cone_windows_at_full_size(mcl):
    """L = 2^17 (2^34 one-bit sites, 2 GiB), the size of the 1-bit benchmark."""
    print("lut full-size windows", flush=True)
    L, seed, n, beta = 2**17, 1004, 6, BETA_C
    lat = mcl.Lattice(LUT, L, seed)
    lat.sweep(n, beta)
    W, pad = 48, 2 * n
    P = W + 2 * pad
    for (x0, y0) in [(0, 0), (L - 24, L - 24), (L // 2 + 7, 12345), (98765, L - 10), (L - 40, 3)]:
        got = lat.read_window(x0, y0, W, W)
        patch = oracle.window_run(LUT, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, beta)
        assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    m = lat.measure(mcl.CORR_PROTOCOL)
    N = L * L
    assert m["invalid"] == 0 and m["counts"][1] == 0 and m["Q"] == N
    assert m["M"] == m["counts"][2] - m["counts"][0]
    assert m["Cx"][0] == N and m["Cy"][0] == N
    assert sum(m["sd"]) == N and sum((k - 4) * v for k, v in enumerate(m["sd"])) == 2 * m["B"]
    assert all(v == 0 for v in m["sd"][1::2])
    assert np.all(np.abs(m["Cx"]) <= m["nsrc"]) and np.all(np.abs(m["Cy"]) <= m["nsrc"])
    assert np.all(m["Cx"][1:8] > 0) and np.all(m["Cy"][1:8] > 0)
    lat.free()
