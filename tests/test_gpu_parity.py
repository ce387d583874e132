"""GPU vs oracle, bit-exact: lattices after n sweeps, and the integer
measurement sums, through the C ABI on the same seeded inputs.  Sizes span
one to many 16-byte columns per row (L = 64 is a single column), non-power-
of-two L, and every temperature regime including beta = infinity."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2
INF = float("inf")


@pytest.fixture(scope="module")
def mcl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_18624_amd as m
    m.lib()
    return m


def _oracle_run(model, L, seed, init, n, beta, D, t0=0, start=None):
    s = oracle.init(model, L, seed, init) if start is None else start.copy()
    if n:
        oracle.sweep(s, model, seed, t0, n, beta, D)
    return s


@pytest.mark.parametrize("model,init", [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2), (1, 3)])
@pytest.mark.parametrize("L", [64, 192, 256])
def test_init_parity(mcl, model, init, L):
    print("init parity", model, init, L, flush=True)
    lat = mcl.Lattice(model, L, 1001 + L, init)
    assert np.array_equal(lat.read(), oracle.init(model, L, 1001 + L, init))


ISING_CASES = [
    (64, 1, 1, BETA_C / 0.9), (64, 2, 17, BETA_C), (128, 3, 3, BETA_C / 0.5), (256, 1001, 17, BETA_C / 0.9),
    (256, 5, 2, INF), (192, 6, 5, BETA_C / 1.5), (512, 7, 3, BETA_C), (1024, 8, 2, BETA_C / 0.9),
    (320, 9, 4, 0.0),
]


@pytest.mark.parametrize("L,seed,n,beta", ISING_CASES)
def test_ising_sweep_parity(mcl, L, seed, n, beta):
    print("ising sweep parity", L, seed, n, beta, flush=True)
    lat = mcl.Lattice(mcl.ISING, L, seed)
    lat.sweep(n, beta)
    got = lat.read()
    want = _oracle_run(0, L, seed, 0, n, beta, 0.0)
    assert lat.t == n
    assert np.array_equal(got, want), "mismatch at %d cells" % int((got != want).sum())


BC_CASES = [
    (64, 11, 1, 1 / 1.4, 1.0), (64, 12, 17, 0.6, 0.0), (128, 13, 3, 1.0, 0.5), (256, 1003, 5, 1 / 1.4, 1.0),
    (256, 14, 3, INF, 1.0), (192, 15, 4, 0.5, -3.0), (512, 16, 2, 0.8, 0.5), (1024, 17, 2, 1 / 1.4, 1.0),
    (128, 18, 3, 0.0, 2.0),
]


@pytest.mark.parametrize("L,seed,n,beta,D", BC_CASES)
def test_bc_sweep_parity(mcl, L, seed, n, beta, D):
    print("bc sweep parity", L, seed, n, beta, D, flush=True)
    lat = mcl.Lattice(mcl.BC, L, seed)
    lat.sweep(n, beta, D)
    got = lat.read()
    want = _oracle_run(1, L, seed, 0, n, beta, D)
    assert np.array_equal(got, want), "mismatch at %d cells" % int((got != want).sum())


@pytest.mark.parametrize("model", [0, 1])
def test_split_calls_and_restart(mcl, model):
    """n sweeps in pieces, and a restore from a host copy at t0, equal the
    oracle's uninterrupted run."""
    print("split/restart", model, flush=True)
    L, seed, beta, D = 128, 77, BETA_C / 0.9, 0.5
    a = mcl.Lattice(model, L, seed)
    for n in (3, 1, 13):
        a.sweep(n, beta, D)
    want = _oracle_run(model, L, seed, 0, 17, beta, D)
    assert np.array_equal(a.read(), want)
    # checkpoint at t = 17, restore into a fresh handle, continue
    snap, t = a.read(), a.t
    b = mcl.Lattice(model, L, seed)
    b.write(snap, t)
    b.sweep(5, beta, D)
    a.sweep(5, beta, D)
    assert np.array_equal(a.read(), b.read())
    assert np.array_equal(b.read(), _oracle_run(model, L, seed, 0, 5, beta, D, t0=17, start=snap))
    # packed checkpoint
    c = mcl.Lattice(model, L, seed)
    c.write_packed(a.read_packed(), a.t)
    c.sweep(2, beta, D)
    a.sweep(2, beta, D)
    assert np.array_equal(a.read(), c.read())


def test_write_arbitrary_state(mcl):
    rng = np.random.default_rng(5)
    for model, vals in ((0, [-1, 1]), (1, [-1, 0, 1])):
        s = rng.choice(vals, size=(128, 128)).astype(np.int8)
        lat = mcl.Lattice(model, 128, 3)
        lat.write(s, 40)
        assert np.array_equal(lat.read(), s)
        lat.sweep(3, 0.7, 0.3)
        assert np.array_equal(lat.read(), _oracle_run(model, 128, 3, 0, 3, 0.7, 0.3, t0=40, start=s))
    with pytest.raises(mcl.MclError):
        mcl.Lattice(0, 64, 1).write(np.zeros((64, 64), dtype=np.int8), 0)   # 0 is not an Ising spin


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


@pytest.mark.parametrize("model,L,n", [(0, 64, 3), (0, 256, 8), (1, 128, 4), (1, 192, 2), (0, 320, 1)])
def test_measure_full_parity(mcl, model, L, n):
    print("measure full", model, L, n, flush=True)
    lat = mcl.Lattice(model, L, 4242)
    lat.sweep(n, BETA_C / 0.9, 1.0)
    _check_measure(mcl, lat, mcl.CORR_FULL)


@pytest.mark.parametrize("model,L,n", [(0, 64, 1), (0, 256, 16), (1, 512, 4), (0, 1024, 8), (1, 2048, 2)])
def test_measure_protocol_parity(mcl, model, L, n):
    print("measure protocol", model, L, n, flush=True)
    lat = mcl.Lattice(model, L, 99)
    lat.sweep(n, BETA_C, 1.0)
    _check_measure(mcl, lat, mcl.CORR_PROTOCOL)
    _check_measure(mcl, lat, mcl.CORR_NONE)


def test_measure_structured_states(mcl):
    """Closed forms through the device path: ordered states."""
    L = 256
    for model, init, val in ((0, 1, 1), (0, 2, -1), (1, 3, 0)):
        lat = mcl.Lattice(model, L, 0, init)
        m = lat.measure(mcl.CORR_PROTOCOL)
        N = L * L
        assert m["M"] == val * N and m["Q"] == abs(val) * N and m["B"] == 2 * N * val * val
        assert m["sd"] == ([0] * 8 + [N] if val else [0] * 4 + [N] + [0] * 4)
        assert np.array_equal(m["Cx"], abs(val) * m["nsrc"]) and np.array_equal(m["Cy"], abs(val) * m["nsrc"])


def _tuning(mcl, rows=None, graph=0, largest=1, wg=0, split=0, gsweeps=32):
    from paper_2502_18624_amd._lib import GroupTuning
    import ctypes
    t = GroupTuning()
    mcl.lib().mcl_group_tuning_get(ctypes.byref(t))
    if rows is not None:
        for k in range(21):
            t.rows_log2L[k] = rows
    t.use_graph = graph
    t.largest_first = largest
    t.wg_per_cu = wg
    t.split_models = split
    t.graph_sweeps = gsweeps
    assert mcl.lib().mcl_group_tuning_set(ctypes.byref(t)) == 0
    return t


@pytest.mark.parametrize("rows,graph,largest,wg,split,gsweeps", [
    (8, 0, 1, 0, 0, 32), (16, 1, 0, 2, 1, 2), (32, 1, 1, 1, 0, 3), (64, 0, 0, 8, 1, 32), (16, 1, 1, 4, 0, 1)])
def test_group_sweep_tunings_are_bit_identical(mcl, rows, graph, largest, wg, split, gsweeps):
    """Every tuning of the batched path gives the plain path's lattices: the
    draws are keyed by the logical site, never by the launch shape.  The
    group mixes all three models; three calls of the same shape run plain,
    then capture a graph, then replay it (graph tunings)."""
    print("group tuning", rows, graph, largest, wg, split, gsweeps, flush=True)
    import ctypes
    from paper_2502_18624_amd._lib import GroupTuning
    saved = GroupTuning()
    mcl.lib().mcl_group_tuning_get(ctypes.byref(saved))
    try:
        _tuning(mcl, rows, graph, largest, wg, split, gsweeps)
        rng = np.random.default_rng(rows + 10 * graph + 100 * largest + 1000 * wg)
        specs = []
        for i in range(9):
            model = int(rng.integers(0, 3))
            L = int(rng.choice([256, 512, 768] if model == 2 else [64, 128, 192, 256, 512]))
            n = int(rng.integers(0, 5))                     # n = 0: left untouched
            specs.append((model, L, 3000 + i, n, float(rng.uniform(0.5, 1.5)) * BETA_C,
                          float(rng.choice([0.0, 0.5, 1.0]))))
        lats = [mcl.Lattice(m, L, sd) for (m, L, sd, _, _, _) in specs]
        for rep in range(3):                                 # plain, capture, replay
            mcl.group_sweep(lats, [sp[3] for sp in specs], [sp[4] for sp in specs], [sp[5] for sp in specs])
        for lat, (m, L, sd, n, b, D) in zip(lats, specs):
            assert lat.t == 3 * n
            want = _oracle_run(m, L, sd, 0, 3 * n, b, D)
            assert np.array_equal(lat.read(), want), (m, L, n)
    finally:
        mcl.lib().mcl_group_tuning_set(ctypes.byref(saved))


def test_group_sweep_rejects_mixed_streams(mcl):
    import torch
    a = mcl.Lattice(0, 64, 1)
    b = mcl.Lattice(0, 64, 2, stream=torch.cuda.Stream())
    with pytest.raises(mcl.MclError):
        mcl.group_sweep([a, b], [1, 1], [0.5, 0.5])


def test_group_sweep_rejects_shared_memory(mcl):
    """The same handle twice, or two handles on one device buffer, both
    with work in one call: rejected before anything is queued.  An entry
    with no work may share memory with another."""
    print("group shared memory", flush=True)
    L, beta = 128, BETA_C
    a = mcl.Lattice(0, L, 31)
    before = a.read()
    with pytest.raises(mcl.MclError):
        mcl.group_sweep([a, a], [2, 1], [beta, beta])
    assert a.t == 0 and np.array_equal(a.read(), before)
    b = mcl.Lattice(0, L, 32, mem=a.mem)                # b's initial state now fills the buffer
    with pytest.raises(mcl.MclError):
        mcl.group_sweep([a, b], [1, 1], [beta, beta])
    assert a.t == 0 and b.t == 0
    mcl.group_sweep([a, b], [2, 0], [beta, beta])
    assert a.t == 2 and b.t == 0
    want = _oracle_run(0, L, 31, 0, 2, beta, 0.0, start=oracle.init(0, L, 32))
    assert np.array_equal(a.read(), want)


def test_group_sweep_equals_plain(mcl):
    rng = np.random.default_rng(3)
    specs = []
    for i in range(6):
        model = i % 2
        L = int(rng.choice([64, 128, 256]))
        specs.append((model, L, 2000 + i, int(rng.integers(1, 6)), float(rng.uniform(0.5, 1.5)) * BETA_C,
                      float(rng.choice([0.0, 0.5, 1.0]))))
    lats = [mcl.Lattice(m, L, s) for (m, L, s, _, _, _) in specs]
    mcl.group_sweep(lats, [sp[3] for sp in specs], [sp[4] for sp in specs], [sp[5] for sp in specs])
    for lat, (m, L, s, n, b, D) in zip(lats, specs):
        assert lat.t == n
        assert np.array_equal(lat.read(), _oracle_run(m, L, s, 0, n, b, D))


@pytest.mark.parametrize("budget,model", [(500, 0), (200, 0), (500, 1), (300, 1), (500, 2), (200, 2)])
def test_sampled_x_correlation_in_residue_passes(mcl, monkeypatch, budget, model):
    """The x-correlation of the sampled sources keeps the source row and a
    group of residue rows in LDS as bits; lattices whose rows do not fit
    (Blume-Capel at L = 2^20) take several passes.  Forcing a small LDS
    budget runs that form at L = 4096 (rows of 32 bytes a bit plane, each
    residue row stored twice and padded by 8 bytes; 500 bytes: 4 residues
    per pass for Ising, 2 for Blume-Capel; 200 for Ising and 300 for
    Blume-Capel: one), against the oracle.  The distance list takes one
    launch per 512 distances, several at t = 10^6 (below)."""
    print("sampled x in passes", budget, model, flush=True)
    monkeypatch.setenv("MCL_SX_LDS_BUDGET", str(budget))
    L = 4096
    lat = mcl.Lattice(model, L, 31 + model)
    lat.sweep(3, BETA_C, 1.0)
    s = lat.read()
    m = lat.measure(mcl.CORR_PROTOCOL)
    Cx, Cy, ns = oracle.corr(s, oracle.CORR_PROTOCOL, m["r"])
    assert np.array_equal(m["Cx"], Cx) and np.array_equal(m["Cy"], Cy)


def test_free_waits_for_the_lattice_stream(mcl):
    """A lattice whose buffer was allocated on the current stream but whose
    sweeps run on a side stream, freed right after queuing them: the buffer
    goes back to the caching allocator only once the sweeps have run, so a
    tensor allocated and filled at once keeps its values."""
    import torch
    print("free waits for the stream", flush=True)
    side = torch.cuda.Stream()
    for L in (8192, 2048):                   # plain launches; graph replays (L <= 4096, 32-sweep chunks)
        lat = mcl.Lattice(0, L, 91, stream=side)
        nbytes = lat.mem.numel()
        torch.cuda.synchronize()
        lat.sweep(64, BETA_C)
        lat.free()
        x = torch.full((nbytes,), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        assert int((x != 7).sum()) == 0, L
        del x


def test_lattices_on_separate_streams(mcl):
    """Independent handles on their own streams, their sweeps queued
    interleaved and running concurrently: each ends equal to the oracle."""
    import torch
    print("separate streams", flush=True)
    streams = [torch.cuda.Stream() for _ in range(3)]
    specs = [(0, 512, 61, BETA_C, 0.0), (1, 256, 62, 1 / 1.4, 1.0), (2, 512, 63, BETA_C / 0.9, 0.0)]
    lats = [mcl.Lattice(m, L, sd, stream=st) for (m, L, sd, _, _), st in zip(specs, streams)]
    for _ in range(3):
        for lat, (m, L, sd, b, D) in zip(lats, specs):
            lat.sweep(2, b, D)
    torch.cuda.synchronize()
    for lat, (m, L, sd, b, D) in zip(lats, specs):
        assert lat.t == 6
        assert np.array_equal(lat.read(), _oracle_run(m, L, sd, 0, 6, b, D)), m


def _band_rows(model, L):
    """Rows per thread of the plain half-sweep: 32, halved (down to 2)
    until a launch has 2^20 threads; a thread owns one 16-byte column."""
    Q = L // (256 if model == 2 else 64)
    rows = 32
    while rows > 2 and Q * (L // rows) < 2**20:
        rows //= 2
    return rows


# sizes at which the plain sweep takes each band height, both cell widths
BAND_CASES = [(0, 2**13, 2), (1, 2**14, 4), (0, 24576, 8), (1, 2**15, 16), (2, 2**15, 4), (2, 49152, 8),
              (2, 2**16, 16)]


@pytest.mark.parametrize("model,L,rows", BAND_CASES)
def test_band_heights(mcl, model, L, rows):
    """Light-cone windows straddling band boundaries (first, middle and
    last band, both horizontal wraps) after 3 sweeps, against the oracle."""
    assert _band_rows(model, L) == rows
    print("band heights", model, L, rows, flush=True)
    n, seed = 3, 2201 + model
    beta, D = (1 / 1.4, 1.0) if model == 1 else (BETA_C, 0.0)
    lat = mcl.Lattice(model, L, seed)
    lat.sweep(n, beta, D)
    W, pad = 32, 2 * n
    P = W + 2 * pad
    ys = [L - W // 2, rows * (L // rows // 2) - W // 2, L - rows - W // 2]
    for y0 in ys:
        for x0 in (0, L // 3, L - 16):
            got = lat.read_window(x0, y0 % L, W, W)
            patch = oracle.window_run(model, L, seed, (x0 - pad) % L, (y0 - pad) % L, P, n, beta, D)
            assert np.array_equal(got, patch[pad:pad + W, pad:pad + W]), (x0, y0)
    lat.free()


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("L", [512, 4096])
def test_counts_report_cells_that_hold_no_spin(mcl, model, L):
    """A packed lattice with some nibbles set to values no spin has (3 .. 15,
    and 1, the Blume-Capel zero, in an Ising lattice): the +1 / 0 / -1
    counts and the invalid count equal those of the cells as written.  At
    L = 4096 with correlations, where the short-distance tiles of 4-bit
    Ising cells take over the B/M/Q pass, such cells send the pass back to
    its own kernel: every sum but the correlations is the one without them."""
    print("invalid cells", model, L, flush=True)
    lat = mcl.Lattice(model, L, 77 + model)
    buf = lat.read_packed().copy()
    rng = np.random.default_rng(5 + model)
    pos = rng.choice(buf.size, size=300, replace=False)
    vals = rng.integers(1, 16, size=(300, 2))
    for p, (lo, hi) in zip(pos, vals):
        buf[p] = (int(hi) << 4) | int(lo)
    lat.write_packed(buf, 0)
    m = lat.measure(mcl.CORR_NONE)
    nib = np.concatenate([buf & 15, buf >> 4])
    want = [int((nib == 0).sum()), int((nib == 1).sum()), int((nib == 2).sum())]
    assert m["counts"] == want
    assert m["invalid"] == int((nib > 2).sum()) > 0
    assert sum(m["counts"]) + m["invalid"] == L * L
    if L >= 4096:
        mc = lat.measure(mcl.CORR_PROTOCOL)
        for k in ("B", "M", "Q", "counts", "invalid", "sd"):
            assert mc[k] == m[k], k
