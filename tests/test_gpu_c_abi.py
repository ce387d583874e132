"""The C program tests/c_abi_quench.c drives the library through include/mcl.h
alone (hipMalloc'd buffer, null stream, no Python in the process); its
integer output equals the oracle's."""
import math
import os
import subprocess

import pytest

import oracle

pytestmark = pytest.mark.gpu

BETA_C = math.log(1 + math.sqrt(2)) / 2


@pytest.fixture(scope="module")
def binary():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import c_abi
    return c_abi.BIN if os.path.exists(c_abi.BIN) else c_abi.build()


@pytest.mark.parametrize("model,L,seed,n,beta,D", [
    (0, 1024, 5, 20, BETA_C, 0.0), (1, 512, 6, 12, 1 / 1.4, 1.0), (2, 1024, 7, 16, BETA_C, 0.0),
])
def test_c_program_equals_oracle(binary, model, L, seed, n, beta, D):
    print("C program", model, L, flush=True)
    out = subprocess.run([binary, str(model), str(L), str(seed), str(n), repr(beta), repr(D)], check=True,
                         capture_output=True, text=True, timeout=120).stdout.split()
    v = [int(x) for x in out]
    s = oracle.init(model, L, seed)
    oracle.sweep(s, model, seed, 0, n, beta, D, nthreads=4)
    om = oracle.measure(s)
    r = oracle.rset(oracle.CORR_PROTOCOL, L, n)
    Cx, Cy, _ = oracle.corr(s, oracle.CORR_PROTOCOL, r)
    assert v[:7] == [n, om["B"], om["M"], om["Q"], *om["counts"]]
    assert v[7:16] == list(oracle.sd_hist(s))
    assert v[16:] == [int(Cx[1]), int(Cy[1]), len(r)]
