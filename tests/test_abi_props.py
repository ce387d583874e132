"""Property tests of the library's host-side tables and distance sets
against the oracle over randomly drawn arguments (CPU; the library is
loaded but no device call is made)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def mcl():
    import paper_2502_18624_amd as m
    m.lib()
    return m


betas = st.one_of(st.floats(min_value=0.0, max_value=60.0, allow_nan=False), st.just(float("inf")),
                  st.sampled_from([0.0, 0.44068679350977147, 0.5, 1 / 1.4]))


@SETTINGS
@given(beta=betas)
def test_ising_thresholds(mcl, beta):
    assert mcl.thresholds(mcl.ISING, beta) == oracle.ising_thresholds(beta)


@SETTINGS
@given(beta=betas, D=st.floats(min_value=-8.0, max_value=8.0, allow_nan=False))
def test_bc_table(mcl, beta, D):
    thr, alw = mcl.thresholds(mcl.BC, beta, D)
    othr, oalw = oracle.bc_table(beta, D)
    assert np.array_equal(thr.reshape(3, 2, 9).astype(np.uint64), othr)
    assert np.array_equal(alw.reshape(3, 2, 9), oalw)


@SETTINGS
@given(beta=betas)
def test_lut_table(mcl, beta):
    T = mcl.lut_table(beta)
    assert T == oracle.lut_table(beta)
    assert T[0] == 0 and all(a <= b for a, b in zip(T, T[1:])) and T[-1] <= 2**32


@SETTINGS
@given(k=st.integers(min_value=6, max_value=20), t=st.integers(min_value=0, max_value=2**32))
def test_protocol_distances(mcl, k, t):
    L = 2**k
    r = mcl.rset(mcl.CORR_PROTOCOL, L, t)
    assert np.array_equal(r, oracle.rset(oracle.CORR_PROTOCOL, L, t))
    assert r[0] == 0 and np.all(np.diff(r) > 0) and r[-1] <= L // 2


@SETTINGS
@given(m=st.integers(min_value=1, max_value=64))
def test_full_distances(mcl, m):
    L = 64 * m
    assert np.array_equal(mcl.rset(mcl.CORR_FULL, L), np.arange(L // 2 + 1))
    assert np.array_equal(mcl.rset(mcl.CORR_FULL, L), oracle.rset(oracle.CORR_FULL, L))


@SETTINGS
@given(model=st.sampled_from([0, 1, 2]), m=st.integers(min_value=1, max_value=4096))
def test_footprint_covers_the_planes(mcl, model, m):
    q = 256 if model == 2 else 64
    L = q * m
    if L > 2**20:
        return
    bits = 1 if model == 2 else 4
    nb = mcl.query_bytes(model, L)
    # both planes and the bits of the sampled columns (two bit planes for
    # Blume-Capel; for 4-bit Ising room for the residue rows of the sampled
    # rows besides), ceil(L / 512) words a row
    base = L * L * bits // 8 + (1 if model == 2 else 2) * L * 4 * max(1, -(-L // 512))
    assert base <= nb <= base + 64 * L + 8192 + (32768 if model == 2 else 0)
