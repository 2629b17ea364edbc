"""Three-way pin of d loss / d kappa: adjoint solves, central differences, eigen-expansion."""
import numpy as np
import pytest

from oracle import assembly, evaluate, geometry, gradient, noise
from paper_2605_24882_amd import inputs


@pytest.fixture(scope="module")
def setup():
    d = assembly.Discretisation(3, 1)
    pts, y = inputs.sphere_points_and_targets(40, seed=7)
    patch, s, t = geometry.invert(pts)
    Phi = evaluate.phi_matrix(d, patch, s, t)
    b = noise.load(d, inputs.noise_vectors([0, 1], inputs.noise_length(3, 1)))
    return d, Phi, y, b


def test_phi_interpolates_smooth_function(setup):
    d, Phi, y, b = setup
    # a degree-p spline reproduces the constant 1 and the coordinate functions only approximately;
    # the constant is reproduced exactly (partition of unity)
    assert np.allclose(Phi @ np.ones(d.N), 1.0, atol=1e-14)


@pytest.mark.parametrize("beta", [0.8, 1.6, 2.3])
def test_adjoint_fd_and_eigen_agree(setup, beta):
    d, Phi, y, b = setup
    kappa, h, K = 3.0, 0.4, 12
    g_adj, u = gradient.adjoint(d.M, d.S, kappa, beta, h, K, K, b, Phi, y)
    g_eig, ue = gradient.eigen_expansion(d.M, d.S, kappa, beta, h, K, K, b, Phi, y)
    g_fd = gradient.finite_difference(d.M, d.S, kappa, beta, h, K, K, b, Phi, y, delta=1e-5)
    assert np.allclose(u, ue, rtol=1e-11, atol=1e-14 * np.abs(u).max())
    assert np.allclose(g_adj, g_eig, rtol=1e-9)
    assert np.allclose(g_adj, g_fd, rtol=1e-6)


@pytest.mark.parametrize("beta", [0.8, 2.3])
def test_two_pass_adjoint_fd_and_eigen_agree(setup, beta):
    """Improved split (the rule applied twice: beta' > 2/3 at 0.8, beta' < 1/3 at 2.3): the backward
    passes of the adjoint against central differences of the two-pass sampler and the dense
    eigen-expansion of lam^-n Q(lam)^2."""
    d, Phi, y, b = setup
    kappa, h, K = 3.0, 0.4, 12
    g_adj, u = gradient.adjoint_two_pass(d.M, d.S, kappa, beta, h, K, K, b, Phi, y)
    g_eig, ue = gradient.eigen_expansion(d.M, d.S, kappa, beta, h, K, K, b, Phi, y, mode="improved")
    g_fd = gradient.finite_difference(d.M, d.S, kappa, beta, h, K, K, b, Phi, y, delta=1e-5, mode="improved")
    assert np.allclose(u, ue, rtol=1e-11, atol=1e-14 * np.abs(u).max())
    assert np.allclose(g_adj, g_eig, rtol=1e-9)
    assert np.allclose(g_adj, g_fd, rtol=1e-6)
