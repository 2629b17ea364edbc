"""Pins of the oracle's point evaluation Phi (Sec. 2.3: the value of a field of S^0_{j,p} at the
surface point F_m(s, t) is the tensor spline sum of its patch coefficients at (s, t)).

Phi is checked against functions the paper's spaces contain or approximate, so a transposed
parameter pair, a transposed coefficient grid or a wrong patch shows up as a wrong value:
  * on the flat unit square (the identity map, one patch) the L2 projection of x^2 y, which lies in
    S_{j,p} for p >= 2, is reproduced exactly at random (s, t); the transposed evaluation gives
    x y^2 instead;
  * on the six-patch sphere the L2 projection of a smooth non-symmetric function converges at the
    points at the spline rate h^(p+1), which no evaluation with a wrong patch, parameter or
    coefficient orientation does.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assembly, evaluate, geometry
from tests.open_surfaces import square


def _project(d, fun, q):
    """Coefficients of the L2 projection M^-1 <fun, phi_i> (eq. mass)."""
    return spla.spsolve(d.M.tocsc(), assembly.load_vector(d, fun, q))


@pytest.mark.parametrize("p", [2, 3])
def test_phi_reproduces_spline_on_flat_square(p):
    surf = geometry.NurbsSurface(*square())
    d = assembly.Discretisation(p, 2, surf)
    c = _project(d, lambda X: X[..., 0] ** 2 * X[..., 1], p + 2)
    rng = np.random.default_rng(3)
    s, t = rng.random(40), rng.random(40)
    s[:4] = [0.0, 1.0, 0.25, 0.5]  # knots and the end points
    t[:4] = [1.0, 0.0, 0.5, 0.75]
    vals = evaluate.phi_matrix(d, np.zeros(40, dtype=int), s, t) @ c
    assert np.allclose(vals, s ** 2 * t, rtol=0, atol=1e-12)
    # the transposed evaluation is a different function (the pin can fail)
    assert not np.allclose(evaluate.phi_matrix(d, np.zeros(40, dtype=int), t, s) @ c, s ** 2 * t, atol=1e-3)


def test_phi_rows_sum_to_one_and_hit_the_right_coefficients():
    """Partition of unity, and at the patch corners (s, t) in {0, 1}^2 the single non-zero basis function
    is the corner coefficient of the patch grid (ix along s, iy along t)."""
    d = assembly.Discretisation(2, 2)
    n1 = d.n1
    for m in range(6):
        s = np.array([0.0, 1.0, 0.0, 1.0])
        t = np.array([0.0, 0.0, 1.0, 1.0])
        Phi = evaluate.phi_matrix(d, np.full(4, m), s, t).toarray()
        expect = [d.l2g[m, 0, 0], d.l2g[m, 0, n1 - 1], d.l2g[m, n1 - 1, 0], d.l2g[m, n1 - 1, n1 - 1]]
        for k in range(4):
            assert Phi[k, expect[k]] == pytest.approx(1.0, abs=1e-15)
            assert np.count_nonzero(np.abs(Phi[k]) > 1e-15) == 1


def test_phi_projection_converges_on_sphere():
    """|Phi P_h f - f| at 200 random sphere points for f = x + 2 y^2 z (no symmetry swaps x, y, z):
    the error falls by about 2^(p+1) per level (p = 2)."""
    p = 2

    def fun(X):
        return X[..., 0] + 2.0 * X[..., 1] ** 2 * X[..., 2]

    rng = np.random.default_rng(11)
    pts = rng.standard_normal((200, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    patch, s, t = geometry.invert(pts)
    errs = []
    for j in (2, 3, 4):
        d = assembly.Discretisation(p, j)
        c = _project(d, fun, p + 3)
        errs.append(np.max(np.abs(evaluate.phi_matrix(d, patch, s, t) @ c - fun(pts))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-3, errs
    assert min(rates) > p + 1 - 0.5, (errs, rates)
    # the evaluation with s and t exchanged does not converge (the pin can fail)
    assert np.max(np.abs(evaluate.phi_matrix(d, patch, t, s) @ c - fun(pts))) > 0.1
