"""Pins of the oracle's NURBS surfaces (Sec. 2.2, definition of the geometry), on the 4 x 4 patch
torus with R = 2, r = 1 (every corner joins four patches):
  - every point of every patch map lies on the torus, (sqrt(x^2 + y^2) - R)^2 + z^2 = r^2;
  - complex-step derivatives of the rational map against central differences;
  - the glued space of a doubly periodic 4 x 4 patch grid has 16 (n - 1)^2 unknowns;
  - 1^T M 1 = area = 4 pi^2 R r, at the rate h^(2p+2) of the Gauss rule;
  - S 1 = 0 and S, M symmetric, M positive definite;
  - the Dirichlet energy of the L2 projection of the height z tends to the integral of
    |grad_Gamma z|^2 = cos^2(phi) over the torus, 2 pi^2 R r;
  - the constant load M 1 gives u = kappa^-2n Q(kappa^2) 1 through the whole sampler.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assembly, fractional, geometry, sinc
from paper_2605_24882_amd import inputs

R, RR = 2.0, 1.0


@pytest.fixture(scope="module")
def torus():
    return geometry.NurbsSurface(*inputs.torus_patches(R, RR))


def test_points_lie_on_the_torus(torus):
    rng = np.random.default_rng(3)
    s, t = rng.random(200), rng.random(200)
    assert torus.npatch == 16
    for m in range(16):
        X = geometry.patch_map(m, s, t, torus)
        err = np.abs((np.hypot(X[:, 0], X[:, 1]) - R) ** 2 + X[:, 2] ** 2 - RR ** 2).max()
        assert err <= 1e-13


def test_complex_step_matches_central_difference(torus):
    s, t = np.array([0.3, 0.71]), np.array([0.55, 0.12])
    for m in (0, 7, 13):
        ds, dt = geometry.jacobian(m, s, t, torus)
        e = 1e-6
        fd_s = (geometry.patch_map(m, s + e, t, torus) - geometry.patch_map(m, s - e, t, torus)) / (2 * e)
        fd_t = (geometry.patch_map(m, s, t + e, torus) - geometry.patch_map(m, s, t - e, torus)) / (2 * e)
        assert np.abs(ds - fd_s).max() <= 1e-8 and np.abs(dt - fd_t).max() <= 1e-8


@pytest.mark.parametrize("p,j", [(1, 2), (2, 2), (2, 3), (3, 2)])
def test_dof_count_and_operators(torus, p, j):
    d = assembly.Discretisation(p, j, torus)
    n = 2 ** j + p
    assert d.N == 16 * (n - 1) ** 2
    one = np.ones(d.N)
    assert np.abs(d.S @ one).max() <= 1e-12
    assert abs(d.M - d.M.T).max() <= 1e-15 and abs(d.S - d.S.T).max() <= 1e-13
    assert np.linalg.eigvalsh(d.M.toarray()).min() > 0


def test_area_converges_at_the_quadrature_rate(torus):
    area = 4 * math.pi ** 2 * R * RR
    errs = []
    for j in (2, 3, 4):
        d = assembly.Discretisation(2, j, torus)
        one = np.ones(d.N)
        errs.append(abs(one @ (d.M @ one) - area))
    assert errs[-1] <= 1e-9 * area
    # h^(2p+2) = 2^-6 per level for p = 2
    assert errs[0] / errs[1] > 40 and errs[1] / errs[2] > 40


def test_dirichlet_energy_of_the_height(torus):
    exact = 2 * math.pi ** 2 * R * RR
    errs = []
    for j in (2, 3, 4):
        d = assembly.Discretisation(2, j, torus)
        f = assembly.load_vector(d, lambda X: X[..., 2], 6)
        u = spla.spsolve(d.M.tocsc(), f)
        errs.append(abs(u @ (d.S @ u) - exact) / exact)
    assert errs[-1] <= 1e-4 and errs[0] > errs[1] > errs[2]


def test_constant_load_closed_form_on_the_torus(torus):
    d = assembly.Discretisation(2, 2, torus)
    kappa, beta, h, K = 3.0, 1.3, 0.4, 12
    b = d.M @ np.ones(d.N)
    u = fractional.sample(d.M, d.S, kappa, beta, h, K, K, b[None, :])[0]
    n, bf = fractional.split_plain(beta)
    expect = kappa ** (-2 * n) * sinc.sinc_sum(kappa ** 2, bf, h, K, K)
    assert np.abs(u - expect).max() <= 1e-11 * abs(expect)


# ---- open surfaces: boundary edges with the natural condition
from tests import open_surfaces  # noqa: E402


@pytest.mark.parametrize("name,lx", [("square", 1.0), ("strip", 2.0)])
def test_open_flat_surfaces_have_the_neumann_spectrum(name, lx):
    """Flat patches with unmatched edges: area, S 1 = 0, and the discrete pencil (S, M) against the
    Neumann eigenvalues of the rectangle (error falling with refinement)."""
    import scipy.linalg as sla
    surf = geometry.NurbsSurface(*getattr(open_surfaces, name)())
    exact = open_surfaces.neumann_eigenvalues(lx, 8)
    errs = []
    for j in (3, 4):
        d = assembly.Discretisation(2, j, surf)
        n1 = 2 ** j + 2
        assert d.N == (n1 if name == "square" else 2 * n1 - 1) * n1
        one = np.ones(d.N)
        assert abs(one @ (d.M @ one) - lx) <= 1e-13 * lx
        assert np.abs(d.S @ one).max() <= 1e-12
        ev = sla.eigh(d.S.toarray(), d.M.toarray(), eigvals_only=True)[:8]
        errs.append(np.abs(ev[1:] - exact[1:]).max() / exact[-1])
        assert abs(ev[0]) <= 1e-10
    assert errs[1] <= 1e-4 and errs[1] < errs[0] / 8
