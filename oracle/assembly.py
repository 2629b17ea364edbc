"""Galerkin matrices of the shifted Laplace-Beltrami problem (oracle, test infrastructure only).

Sec. 2.3 (spaces S^0_{j,p}), Sec. 3.1 (eq. FEM: mass M, stiffness S) and
Sec. 3.2 (pull-back to the reference square, eq. mass and eq. stiffness):

    M_ij = sum_m int a_m phi_i phi_j,
    S_ij = sum_m int grad phi_i^T K_m^{-1} grad phi_j a_m,

with K_m the first fundamental form and a_m = sqrt(det K_m).  The paper leaves
the quadrature open ("appropriately chosen"); the reading used here is tensor
Gauss-Legendre with q = p+1 points per direction and element.

Unknowns: patch-local coefficient grids c[m, iy, ix] (ix along s, iy along t,
n1 = 2^j + p per direction).  Copies of one global unknown on patch interfaces
are identified geometrically: two local coefficients are the same unknown when
their Greville points map to the same surface point (Sec. 2.2 asks only that
neighbouring maps agree up to a rotation, so no orientation is assumed).
Global numbering: scan patches in order, then iy, then ix (ix fastest), and give
the next number to every local coefficient whose surface point is new.
"""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import bspline, geometry


def gauss_legendre_01(q):
    """q-point Gauss-Legendre nodes and weights on [0, 1] (numpy.polynomial.legendre)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return (x + 1.0) / 2.0, w / 2.0


def n_dofs_formula(p, j):
    """Unique unknowns of the conforming six-patch cube topology: 6(n-2)^2 + 12(n-2) + 8."""
    n = 2 ** j + p
    return 6 * (n - 2) ** 2 + 12 * (n - 2) + 8


def dofmap(p, j, perturbed=False, tol=1e-12):
    """local_to_global[m, iy, ix] by Greville-point matching; returns (l2g, N)."""
    knots = bspline.dyadic_knots(p, j)
    g = bspline.greville(knots, p)
    n1 = len(g)
    pts = []
    for m in range(geometry.npatch(perturbed)):
        S, T = np.meshgrid(g, g, indexing="xy")  # S[iy, ix] = g[ix], T[iy, ix] = g[iy]
        pts.append(geometry.patch_map(m, S, T, perturbed).reshape(-1, 3))
    pts = np.concatenate(pts)
    tree = cKDTree(pts)
    l2g = -np.ones(len(pts), dtype=np.int64)
    nxt = 0
    for i in range(len(pts)):
        if l2g[i] >= 0:
            continue
        l2g[i] = nxt
        for k in tree.query_ball_point(pts[i], tol):
            if k > i:
                l2g[k] = nxt
        nxt += 1
    return l2g.reshape(geometry.npatch(perturbed), n1, n1), nxt


class Discretisation:
    """Everything the oracle needs about S^0_{j,p} on one surface."""

    def __init__(self, p, j, perturbed=False, nquad=None):
        self.p, self.j, self.perturbed = p, j, perturbed
        self.q = p + 1 if nquad is None else nquad
        self.n_el = 2 ** j
        self.knots = bspline.dyadic_knots(p, j)
        self.n1 = bspline.n_basis(self.knots, p)
        self.l2g, self.N = dofmap(p, j, perturbed)
        self._elements()
        self._assemble()

    def _elements(self):
        """Per element: global unknown numbers, quadrature data and local basis tables."""
        p, q, ne = self.p, self.q, self.n_el
        xg, wg = gauss_legendre_01(q)
        # quadrature abscissae of element e: (e + xg)/ne; basis functions e..e+p are non-zero
        xs = ((np.arange(ne)[:, None] + xg[None, :]) / ne).reshape(-1)
        Bfull = bspline.basis(self.knots, p, xs).reshape(ne, q, self.n1)
        Dfull = bspline.basis_derivative(self.knots, p, xs).reshape(ne, q, self.n1)
        self.B1 = np.stack([Bfull[e, :, e:e + p + 1] for e in range(ne)])  # (ne, q, p+1)
        self.D1 = np.stack([Dfull[e, :, e:e + p + 1] for e in range(ne)])
        self.xq, self.wq = xs.reshape(ne, q), wg / ne  # abscissae and weights per element
        nloc = (p + 1) ** 2
        el_dofs, el_M, el_S = [], [], []
        for m in range(geometry.npatch(self.perturbed)):
            for ey in range(ne):
                for ex in range(ne):
                    iy = np.arange(ey, ey + p + 1)
                    ix = np.arange(ex, ex + p + 1)
                    # element-local order (b, a): row b along t, column a along s, a fastest
                    el_dofs.append(self.l2g[m][np.ix_(iy, ix)].reshape(nloc))
            # metric at all quadrature points of the patch
            S_, T_ = np.meshgrid(xs, xs, indexing="xy")  # S_[row over t, col over s]
            k11, k12, k22, a = geometry.first_fundamental_form(m, S_, T_, self.perturbed)
            W = np.outer(np.tile(self.wq, ne), np.tile(self.wq, ne))  # [t-point, s-point]
            det = k11 * k22 - k12 * k12
            g11, g12, g22 = k22 / det, -k12 / det, k11 / det  # K^{-1}
            # the same element integrals for all elements of the patch at once: quadrature arrays
            # reshaped to [ey, ex, qy, qx], basis tables By[ey, qy, b], Bx[ex, qx, a] (eq. mass and
            # eq. stiffness with phi_(b,a) = By Bx, d/ds phi = By Dx, d/dt phi = Dy Bx)
            def per_el(f):
                return f.reshape(ne, q, ne, q).transpose(0, 2, 1, 3)

            wa = per_el(W * a)
            G11, G12, G22 = per_el(g11), per_el(g12), per_el(g22)
            B, D = self.B1, self.D1

            def form(w, Ly, Lx, Ry, Rx):
                """sum over (qy, qx) of w Ly[ey,qy,b] Lx[ex,qx,a] Ry[ey,qy,c] Rx[ex,qx,d] -> [(ey,ex),(b,a),(c,d)]"""
                t = np.einsum("EXyx,Eyb,Xxa,Eyc,Xxd->EXbacd", w, Ly, Lx, Ry, Rx, optimize=True)
                return t.reshape(ne * ne, nloc, nloc)

            el_M.append(form(wa, B, B, B, B))
            el_S.append(form(wa * G11, B, D, B, D) + form(wa * G12, B, D, D, B) + form(wa * G12, D, B, B, D)
                        + form(wa * G22, D, B, D, B))
        self.el_dofs = np.array(el_dofs)
        self.el_M = np.concatenate(el_M)
        self.el_S = np.concatenate(el_S)

    def _assemble(self):
        """Sum element matrices into sparse global M and S (eq. FEM)."""
        nloc = self.el_dofs.shape[1]
        rows = np.repeat(self.el_dofs, nloc, axis=1).reshape(-1)
        cols = np.tile(self.el_dofs, (1, nloc)).reshape(-1)
        self.M = sp.csr_matrix((self.el_M.reshape(-1), (rows, cols)), shape=(self.N, self.N))
        self.S = sp.csr_matrix((self.el_S.reshape(-1), (rows, cols)), shape=(self.N, self.N))


def _patch_quadrature(disc, q):
    """Abscissae and weights of a q-point Gauss rule on every element, flattened per direction."""
    xg, wg = gauss_legendre_01(q)
    ne = disc.n_el
    xs = ((np.arange(ne)[:, None] + xg[None, :]) / ne).reshape(-1)
    return xs, np.tile(wg / ne, ne)


def load_vector(disc, fun, q):
    """f_i = <f, phi_i>_Gamma by a q-point Gauss rule per element direction (eq. FEM, right-hand side).

    `fun` maps surface points (..., 3) to values."""
    xs, ws = _patch_quadrature(disc, q)
    B = bspline.basis(disc.knots, disc.p, xs)  # (points along one direction, n1)
    f = np.zeros(disc.N)
    for m in range(geometry.npatch(disc.perturbed)):
        S_, T_ = np.meshgrid(xs, xs, indexing="xy")
        X = geometry.patch_map(m, S_, T_, disc.perturbed)
        a = geometry.first_fundamental_form(m, S_, T_, disc.perturbed)[3]
        W = np.outer(ws, ws) * a * fun(X)  # [t-point, s-point]
        loc = B.T @ W @ B  # [iy, ix] = sum_t sum_s b_iy(t) W b_ix(s)
        np.add.at(f, disc.l2g[m].reshape(-1), loc.reshape(-1))
    return f


def l2_error(disc, u, fun, q):
    """|| u_h - f ||_{L2(Gamma)} by a q-point Gauss rule per element direction (eq. mass)."""
    xs, ws = _patch_quadrature(disc, q)
    B = bspline.basis(disc.knots, disc.p, xs)
    err2 = 0.0
    for m in range(geometry.npatch(disc.perturbed)):
        S_, T_ = np.meshgrid(xs, xs, indexing="xy")
        X = geometry.patch_map(m, S_, T_, disc.perturbed)
        a = geometry.first_fundamental_form(m, S_, T_, disc.perturbed)[3]
        uh = B @ np.asarray(u)[disc.l2g[m]] @ B.T  # [t, s]
        err2 += np.sum(np.outer(ws, ws) * a * (uh - fun(X)) ** 2)
    return np.sqrt(err2)
