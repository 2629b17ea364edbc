"""Pins of the oracle's square root of the mass matrix (Sec. 3.3, eq. sqrt)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly, sqrt_mass


def test_scalar_rule_converges_to_the_square_root():
    """On [m, Mu] = [0.1, 1] the rule approximates sqrt(lam) with errors 1.5e-3, 6e-7, 9e-14 for
    Khat = 2, 4, 8 (exponential convergence in Khat); the constant read as the complete integral of
    the second kind instead would leave an O(1) error."""
    lam = np.linspace(0.1, 1.0, 91)
    errs = [np.max(np.abs(sqrt_mass.scalar(lam, 0.1, 1.0, k) - np.sqrt(lam))) for k in (2, 4, 8)]
    assert 1e-3 < errs[0] < 2e-3 and 1e-7 < errs[1] < 1e-6 and errs[2] < 1e-12
    # slightly loose bounds still work (the rule is a rational approximation on a wider interval)
    assert np.max(np.abs(sqrt_mass.scalar(lam, 0.05, 2.0, 16) - np.sqrt(lam))) < 1e-10


@pytest.fixture(scope="module")
def c1():
    return assembly.Discretisation(2, 2)


def test_apply_matches_dense_square_root(c1):
    m, Mu = sqrt_mass.dense_bounds(c1.M)
    y = np.random.default_rng(3).standard_normal((2, c1.N))
    f = sqrt_mass.apply(c1.M, y, 16, 0.99 * m, 1.01 * Mu)
    R = sla.sqrtm(c1.M.toarray()).real
    ref = (R @ y.T).T
    assert np.linalg.norm(f - ref) <= 1e-10 * np.linalg.norm(ref)


def test_covariance_is_the_mass_matrix(c1):
    """f = R y with R the rule's matrix: R R^T = M (so f ~ N(0, M) for y ~ N(0, I))."""
    m, Mu = sqrt_mass.dense_bounds(c1.M)
    R = sqrt_mass.apply(c1.M, np.eye(c1.N), 16, 0.99 * m, 1.01 * Mu).T
    Md = c1.M.toarray()
    assert np.allclose(R @ R.T, Md, rtol=0, atol=1e-11 * np.abs(Md).max())
