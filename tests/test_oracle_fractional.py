"""Pins of the oracle's fractional solve: closed forms, brute force and the Matern variance."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assembly, fractional, noise, sinc
from paper_2605_24882_amd import inputs


@pytest.fixture(scope="module")
def c1():
    return assembly.Discretisation(2, 2)  # 6 patches, 4 x 4 elements, p = 2: 152 unknowns


def test_nodes_and_weights_match_scalar_rule():
    sigma, omega, t = fractional.nodes(4.0, 0.75, 0.4, 15, 15)
    assert len(sigma) == 31
    lam = np.array([16.0, 30.0, 1000.0])
    q = np.sum(omega[:, None] / (t[:, None] + lam[None, :]), axis=0)
    assert np.allclose(q, sinc.sinc_sum(lam, 0.75, 0.4, 15, 15), rtol=1e-14)


@pytest.mark.parametrize("beta", [0.75, 1.6, 2.3, 2.0])
def test_constant_load_invariant(c1, beta):
    """b = M 1: constants are an eigenvector with mu = 0, so u = kappa^{-2n} Q(kappa^2) 1."""
    kappa, h, K = 4.0, 0.4, 15
    b = c1.M @ np.ones(c1.N)
    u = fractional.sample(c1.M, c1.S, kappa, beta, h, K, K, b)[0]
    n, bf = fractional.split_plain(beta)
    expect = kappa ** (-2 * n) * (sinc.sinc_sum(kappa ** 2, bf, h, K, K) if bf else 1.0)
    assert np.allclose(u, expect, rtol=1e-12)


def test_dense_eigen_identity_c1(c1):
    """The sinc rule applied with sparse solves equals V diag(G) V^T b to rounding."""
    z = inputs.noise_vectors([0], inputs.noise_length(2, 2))
    b = noise.load(c1, z)
    for beta in (0.75, 1.6, 2.3):
        u = fractional.sample(c1.M, c1.S, 4.0, beta, 0.4, 15, 15, b)
        ud = fractional.dense_quadrature(c1.M, c1.S, 4.0, beta, 0.4, 15, 15, b)
        assert np.linalg.norm(u - ud) <= 1e-12 * np.linalg.norm(ud)


def test_exact_power_within_quadrature_error(c1):
    """u_Q differs from the exact discrete power only by the scalar quadrature error."""
    z = inputs.noise_vectors([0], inputs.noise_length(2, 2))
    b = noise.load(c1, z)
    kappa, beta = 4.0, 0.75
    mu = sla.eigh(c1.S.toarray(), c1.M.toarray(), eigvals_only=True)
    lam = kappa ** 2 + np.maximum(mu, 0)
    scalar_err = np.max(np.abs(sinc.sinc_sum(lam, beta, 0.4, 15, 15) - lam ** -beta) / lam ** -beta)
    uq = fractional.sample(c1.M, c1.S, kappa, beta, 0.4, 15, 15, b)
    ue = fractional.dense_exact(c1.M, c1.S, kappa, beta, b)
    rel = np.linalg.norm(uq - ue) / np.linalg.norm(ue)
    assert rel <= scalar_err * 1.0001
    # and with many more nodes the rule converges to the exact power
    uq2 = fractional.sample(c1.M, c1.S, kappa, beta, 0.1, 200, 600, b)
    assert np.linalg.norm(uq2 - ue) / np.linalg.norm(ue) < 1e-8


def test_integer_beta_is_the_chain(c1):
    """beta = 2: u = A^-1 M A^-1 b (Sec. 3.4 integer case)."""
    b = np.random.default_rng(5).standard_normal(c1.N)
    A = (16.0 * c1.M + c1.S).toarray()
    expect = np.linalg.solve(A, c1.M @ np.linalg.solve(A, b))
    u = fractional.sample(c1.M, c1.S, 4.0, 2.0, 0.4, 15, 15, b)[0]
    assert np.allclose(u, expect, rtol=1e-12, atol=1e-16)


def _series(kappa, beta, L=20000):
    l = np.arange(L, dtype=np.float64)
    return np.sum((2 * l + 1) * (kappa ** 2 + l * (l + 1)) ** (-2 * beta)) / (4 * math.pi)


def _eq_sigma(kappa, beta):
    nu = 2 * beta - 1
    return math.gamma(nu) / math.gamma(nu + 1) / (4 * math.pi) * kappa ** (-2 * nu)


def test_matern_variance():
    """Sec. 1, eq. (sigma) with d = 2: sigma^2 = 1/(4 pi nu kappa^{2 nu}).  The mean discrete
    variance sum_i (kappa^2+mu_i)^{-2 beta} / |Gamma| approaches the sphere's spectral series
    under refinement, and the series approaches eq. (sigma) as kappa grows."""
    kappa, beta = 4.0, 1.6
    ref = _series(kappa, beta)
    errs = []
    for j in (2, 3, 4):
        d = assembly.Discretisation(2, j)
        mu = sla.eigh(d.S.toarray(), d.M.toarray(), eigvals_only=True)
        var = np.sum((kappa ** 2 + np.maximum(mu, 0)) ** (-2 * beta)) / (4 * math.pi)
        errs.append(abs(var - ref) / ref)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.005
    r4 = _series(4.0, 1.6) / _eq_sigma(4.0, 1.6)
    r10 = _series(10.0, 1.6) / _eq_sigma(10.0, 1.6)
    r30 = _series(30.0, 1.6) / _eq_sigma(30.0, 1.6)
    assert r4 > r10 > r30 > 1.0 and r30 < 1.001
    assert r10 == pytest.approx(1.0074, abs=5e-4)


def test_white_noise_factor_reproduces_mass(c1):
    """b = L z with the tall element-wise factor: L L^T = M exactly (Sec. 3.3)."""
    F = noise.factor_matrix(c1)
    assert np.allclose(F @ F.T, c1.M.toarray(), atol=1e-15)
    z = inputs.noise_vectors([3], F.shape[1])
    assert np.allclose(noise.load(c1, z)[0], F @ z[0], atol=1e-15)


@pytest.mark.parametrize("beta,expect", [(0.8, (0, 0.4, 2)), (2.3, (1, 0.65, 2)), (1.5, (1, 0.5, 1)),
                                         (0.2, (0, 0.2, 1)), (2.9, (2, 0.45, 2)), (3.0, (3, 0.0, 1))])
def test_improved_split_rule(beta, expect):
    """Sec. 3.4: beta' < 1/3 -> (n-1) + 2 (beta'+1)/2, beta' > 2/3 -> n + 2 beta'/2, else plain;
    with n = 0 and beta' < 1/3 there is no integer part to borrow from, so the split stays plain."""
    n, bf, passes = fractional.split(beta, "improved")
    assert (n, passes) == expect[::2] and abs(bf - expect[1]) < 1e-14
    assert abs(n + passes * bf - beta) < 1e-14


@pytest.mark.parametrize("beta", [0.8, 2.3, 2.9])
def test_improved_split_constant_load_and_dense_identity(c1, beta):
    """Two passes of the rule: b = M 1 gives kappa^{-2n} Q(kappa^2)^2 1, and a white-noise load gives
    V diag(lam^-n Q(lam)^2) V^T b."""
    kappa, h, K = 4.0, 0.4, 15
    n, bf, passes = fractional.split(beta, "improved")
    assert passes == 2
    u = fractional.sample(c1.M, c1.S, kappa, beta, h, K, K, c1.M @ np.ones(c1.N), mode="improved")[0]
    assert np.allclose(u, kappa ** (-2 * n) * sinc.sinc_sum(kappa ** 2, bf, h, K, K) ** 2, rtol=1e-12)
    b = noise.load(c1, inputs.noise_vectors([3], inputs.noise_length(2, 2)))
    u = fractional.sample(c1.M, c1.S, kappa, beta, h, K, K, b, mode="improved")
    ud = fractional.dense_quadrature(c1.M, c1.S, kappa, beta, h, K, K, b, mode="improved")
    assert np.linalg.norm(u - ud) <= 1e-12 * np.linalg.norm(ud)


@pytest.mark.parametrize("beta", [2.2, 0.9])
def test_improved_split_is_more_accurate_at_equal_solves(c1, beta):
    """The paper's claim behind the modification (Fig. 6): for beta' near 0 or 1 the improved split
    with K/2 nodes per pass is closer to the exact power than the plain split with K nodes, once K is
    in the exponential regime (K = 200 here; at K of a few dozen the plain rule can still win)."""
    z = inputs.noise_vectors([0], inputs.noise_length(2, 2))
    b = noise.load(c1, z)
    kappa, K = 4.0, 200
    ue = fractional.dense_exact(c1.M, c1.S, kappa, beta, b)
    up = fractional.sample(c1.M, c1.S, kappa, beta, 1 / math.sqrt(K), K, K, b)
    ui = fractional.sample(c1.M, c1.S, kappa, beta, 1 / math.sqrt(K // 2), K // 2, K // 2, b, mode="improved")
    ep = np.linalg.norm(up - ue) / np.linalg.norm(ue)
    ei = np.linalg.norm(ui - ue) / np.linalg.norm(ue)
    assert ei < ep, (ei, ep)
