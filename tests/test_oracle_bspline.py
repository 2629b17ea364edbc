"""Pins of the oracle's B-spline, quadrature and knot-insertion routines."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import assembly, bspline


@pytest.mark.parametrize("p,j", [(1, 2), (2, 3), (3, 2), (4, 1), (5, 3)])
def test_basis_matches_scipy_design_matrix(p, j):
    kn = bspline.dyadic_knots(p, j)
    x = np.linspace(0.0, 1.0, 97)
    ours = bspline.basis(kn, p, x)
    ref = BSpline.design_matrix(x, kn, p).toarray()
    assert np.allclose(ours, ref, atol=1e-14)
    assert np.allclose(ours.sum(axis=1), 1.0, atol=1e-14)  # partition of unity


@pytest.mark.parametrize("p,j", [(1, 2), (2, 3), (3, 3), (5, 2)])
def test_derivative_matches_scipy(p, j):
    kn = bspline.dyadic_knots(p, j)
    n = bspline.n_basis(kn, p)
    x = np.random.default_rng(1).uniform(0, 1, 50)
    ours = bspline.basis_derivative(kn, p, x)
    for l in range(n):
        c = np.zeros(n)
        c[l] = 1.0
        ref = BSpline(kn, c, p).derivative()(x)
        assert np.allclose(ours[:, l], ref, atol=1e-11)


def test_dyadic_knot_vector_shape():
    kn = bspline.dyadic_knots(3, 2)
    assert list(kn) == [0, 0, 0, 0, 0.25, 0.5, 0.75, 1, 1, 1, 1]
    assert bspline.n_basis(kn, 3) == 2 ** 2 + 3


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6])
def test_gauss_legendre_exactness(q):
    x, w = assembly.gauss_legendre_01(q)
    for d in range(2 * q):
        assert np.dot(w, x ** d) == pytest.approx(1.0 / (d + 1), rel=1e-13)
    assert np.dot(w, x ** (2 * q)) != pytest.approx(1.0 / (2 * q + 1), rel=1e-10)


@pytest.mark.parametrize("p,j", [(1, 1), (2, 0), (2, 3), (3, 0), (3, 2), (4, 2), (4, 3)])
def test_refinement_matrix(p, j):
    P = bspline.refinement_matrix(p, j)
    assert P.shape == (2 ** (j + 1) + p, 2 ** j + p)
    x = np.random.default_rng(3).uniform(0, 1, 200)
    Bf = bspline.basis(bspline.dyadic_knots(p, j + 1), p, x)
    Bc = bspline.basis(bspline.dyadic_knots(p, j), p, x)
    assert np.allclose(Bf @ P, Bc, atol=1e-13)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0, atol=1e-13)
    if 2 ** j - 1 >= p:
        # a coarse B-spline clear of the repeated end knots (index p .. 2^j - 1) is refined by
        # the uniform subdivision mask 2^-p C(p+1, i)
        c = p
        col = P[:, c]
        nz = col[np.abs(col) > 1e-14]
        mask = np.array([math.comb(p + 1, i) for i in range(p + 2)]) / 2 ** p
        assert np.allclose(nz, mask, atol=1e-13)
