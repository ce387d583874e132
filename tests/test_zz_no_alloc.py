"""group_sweep_noalloc, the batched sweep for callers that cannot allocate,
against group_sweep on twin lattices (same models, sizes, seeds and
parameters): every lattice bit-identical after each of two calls in a row,
the second with a smaller input; a call at the workspace's limit; and the
limit itself reported before anything is queued."""
import math

import numpy as np
import pytest

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


def _planes(lat):
    """The lattice's two colour planes as a device byte tensor."""
    off = lat.ptr - lat.mem.data_ptr()
    nb = lat.L * lat.L * (1 if lat.model == 2 else 4) // 8
    return lat.mem[off:off + nb]


def _same(a, b):
    import torch
    torch.cuda.synchronize()
    return a.t == b.t and bool(torch.equal(_planes(a), _planes(b)))


def _specs(k, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        model = i % 3
        L = int(rng.choice([256, 512, 1024, 2048, 4096]))
        beta = 1.0 / (float(rng.uniform(0.5, 1.5)) / BETA_C)
        D = float(rng.choice([0.0, 0.5, 1.0])) if model == 1 else 0.0
        out.append((model, L, 8100 + i, beta, D))
    return out


def test_noalloc_equals_group_sweep_on_two_calls(mcl):
    print("no-alloc: two calls against group_sweep", flush=True)
    specs = _specs(30, 11)
    specs.append((2, 2 ** 17 + 256, 8200, BETA_C, 0.0))   # above the batched limit: swept on its own
    a = [mcl.Lattice(m, L, sd) for (m, L, sd, _, _) in specs]
    b = [mcl.Lattice(m, L, sd) for (m, L, sd, _, _) in specs]
    betas = [sp[3] for sp in specs]
    Ds = [sp[4] for sp in specs]
    rng = np.random.default_rng(12)
    n1 = [int(rng.integers(1, 5)) for _ in specs]
    mcl.group_sweep(a, n1, betas, Ds, noalloc=True)
    mcl.group_sweep(b, n1, betas, Ds)
    for x, y, sp in zip(a, b, specs):
        assert _same(x, y), sp
    # a smaller second call: fewer replicas, new sweep counts and temperatures,
    # one entry idle; the workspace still holds the first call's image
    k = 7
    n2 = [int(rng.integers(1, 4)) for _ in range(k)]
    n2[3] = 0
    betas2 = [1.0 / (float(rng.uniform(0.5, 1.5)) / BETA_C) for _ in range(k)]
    mcl.group_sweep(a[:k], n2, betas2, Ds[:k], noalloc=True)
    mcl.group_sweep(b[:k], n2, betas2, Ds[:k])
    for x, y, sp in zip(a, b, specs):
        assert _same(x, y), sp
    assert [x.t for x in a[:k]] == [p + q for p, q in zip(n1[:k], n2)]
    for lat in a + b:
        lat.free()


def test_noalloc_limits(mcl):
    print("no-alloc: limits", flush=True)
    beta = 1 / 1.4
    # 1300 Blume-Capel replicas need 1300 x 832 bytes of image: above 1 MiB
    big = [mcl.Lattice(mcl.BC, 64, 9000 + i) for i in range(1300)]
    with pytest.raises(mcl.MclError) as e:
        mcl.group_sweep(big, 1, beta, 1.0, noalloc=True)
    assert e.value.code == -12
    # more than 4096 entries, even with no work
    with pytest.raises(mcl.MclError) as e:
        mcl.group_sweep([big[0]] * 4097, 0, beta, 1.0, noalloc=True)
    assert e.value.code == -12
    assert all(lat.t == 0 for lat in big)
    # 1200 of them fit; the result equals group_sweep's
    twins = [mcl.Lattice(mcl.BC, 64, 9000 + i) for i in range(1200)]
    mcl.group_sweep(big[:1200], 2, beta, 1.0, noalloc=True)
    mcl.group_sweep(twins, 2, beta, 1.0)
    for x, y in zip(big[:1200], twins):
        assert _same(x, y)
    for lat in big + twins:
        lat.free()
