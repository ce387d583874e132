"""The correlation-length estimator xi_{k,k+1} = I_{k+1} / I_k (integrals
of r^k C(r)) against closed forms: for C(r) = exp(-r/a), I_k = k! a^{k+1}, so
xi_{1,2} = 2a and xi_{2,3} = 3a; for C(r) = exp(-(r/a)^2), xi_{1,2} =
(sqrt(pi)/2) a.  The trapezoid rule on the grid of measured distances
(dense, or the protocol's set with its log-spaced tail) reaches them within
its own error bound.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import paper_2502_18624_amd as mcl


@pytest.mark.parametrize("a", [3.0, 20.0, 80.0])
def test_exponential_on_a_dense_grid(a):
    r = np.arange(0, int(60 * a) + 1, dtype=float)
    C = np.exp(-r / a)
    # trapezoid error on a smooth integrand ~ h^2 / (12 a^2) relative, h = 1
    tol = 1.0 / (4 * a * a) + 1e-9
    assert mcl.correlation_length(r, C, 1) == pytest.approx(2 * a, rel=tol)
    assert mcl.correlation_length(r, C, 2) == pytest.approx(3 * a, rel=tol)


@pytest.mark.parametrize("a", [10.0, 50.0])
def test_gaussian_on_a_dense_grid(a):
    r = np.arange(0, int(10 * a) + 1, dtype=float)
    C = np.exp(-(r / a) ** 2)
    assert mcl.correlation_length(r, C, 1) == pytest.approx(math.sqrt(math.pi) / 2 * a, rel=1.0 / (a * a))


@pytest.mark.parametrize("a,t", [(40.0, 1000), (150.0, 4096), (400.0, 2 ** 20)])
def test_exponential_on_the_protocol_distances(a, t):
    """The protocol's r-set at L = 2^17: every r up to r_c(t), then
    floor(2^{x/32}); the coarse tail still integrates to within 1%."""
    L = 2 ** 17
    r = oracle.rset(oracle.CORR_PROTOCOL, L, t).astype(float)
    C = np.exp(-r / a)
    assert mcl.correlation_length(r, C, 1) == pytest.approx(2 * a, rel=1e-2)
    assert mcl.correlation_length(r, C, 2) == pytest.approx(3 * a, rel=1e-2)


def test_scale_covariance_is_exact():
    """Stretching r and the correlation together by lambda multiplies the
    estimate by lambda (the trapezoid rule commutes with the scaling)."""
    r = np.concatenate([np.arange(0, 33.0), np.floor(2.0 ** (np.arange(165, 300) / 32.0))])
    r = np.unique(r)
    C = np.exp(-(r / 17.0) ** 1.5)
    for lam in (2.0, 8.0, 0.5):
        for k in (1, 2):
            assert mcl.correlation_length(lam * r, C, k) == pytest.approx(lam * mcl.correlation_length(r, C, k),
                                                                           rel=1e-12)


def test_cut_at_the_noise_floor():
    """Everything from the first non-positive C on is left out."""
    r = np.arange(0, 200, dtype=float)
    C = np.exp(-r / 10.0)
    noisy = C.copy()
    noisy[120] = -1e-6
    noisy[121:] = np.random.default_rng(1).normal(0.0, 1.0, 79)
    assert mcl.correlation_length(r, noisy, 1) == mcl.correlation_length(r[:120], C[:120], 1)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        mcl.correlation_length([0, 2, 1], [1.0, 0.5, 0.2])
    with pytest.raises(ValueError):
        mcl.correlation_length([0, 1, 2], [1.0, 0.5])
    with pytest.raises(ValueError):
        mcl.correlation_length([0, 1, 2], [1.0, -0.5, 0.2])
