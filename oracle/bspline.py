"""B-splines on p-open dyadic knot vectors (oracle, test infrastructure only).

Sec. 2.1 (definition of p-open knot vectors and the Cox-de Boor recursion)
and Sec. 2.3 (the dyadic knot vectors Xi_{j,p}).  Readings:
  * the first denominator of the recursion is xi_{l+p} - xi_l (the paper's
    typesetting shows xi_j there);
  * a term whose denominator vanishes is dropped (0/0 := 0);
  * the right end point x = 1 belongs to the last non-empty knot span.
"""
import numpy as np


def dyadic_knots(p, j):
    """Xi_{j,p}: p+1 zeros, the interior knots i 2^-j (i = 1..2^j-1), p+1 ones (Sec. 2.3)."""
    n_el = 2 ** j
    interior = [i / n_el for i in range(1, n_el)]
    return np.array([0.0] * (p + 1) + interior + [1.0] * (p + 1))


def n_basis(knots, p):
    """Number of basis functions k = len(Xi) - p - 1 (Sec. 2.1)."""
    return len(knots) - p - 1


def _degree0(knots, x):
    """b_l^0(x) = 1 on [xi_l, xi_{l+1}), x = 1 assigned to the last non-empty span."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(knots) - 1
    B = np.zeros((x.size, m))
    last = max(i for i in range(m) if knots[i] < knots[i + 1])
    for i in range(m):
        inside = (knots[i] <= x) & (x < knots[i + 1])
        if i == last:
            inside = inside | (x == knots[i + 1])
        B[:, i] = inside.astype(np.float64)
    return B


def basis(knots, p, x):
    """Values b_l^p(x) for all l, shape (len(x), k).  Cox-de Boor recursion (Sec. 2.1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    B = _degree0(knots, x)
    for d in range(1, p + 1):
        m = len(knots) - 1 - d
        Bn = np.zeros((x.size, m))
        for l in range(m):
            den1 = knots[l + d] - knots[l]
            den2 = knots[l + d + 1] - knots[l + 1]
            term = np.zeros(x.size)
            if den1 > 0.0:
                term = term + (x - knots[l]) / den1 * B[:, l]
            if den2 > 0.0:
                term = term + (knots[l + d + 1] - x) / den2 * B[:, l + 1]
            Bn[:, l] = term
        B = Bn
    return B


def basis_analytic(knots, p, x):
    """b_l^p(x) for all l with x of any numeric type, complex included (shape (len(x), k)).

    The same recursion as `basis`, with the knot span chosen by the real part of x and the linear
    factors evaluated in x itself, so that the result is the polynomial piece of that span
    continued analytically (used for complex-step derivatives of NURBS maps)."""
    x = np.atleast_1d(np.asarray(x))
    xr = np.real(x)
    m = len(knots) - 1
    B = np.zeros((x.size, m), dtype=np.result_type(x.dtype, np.float64))
    last = max(i for i in range(m) if knots[i] < knots[i + 1])
    for i in range(m):
        inside = (knots[i] <= xr) & (xr < knots[i + 1])
        if i == last:
            inside = inside | (xr == knots[i + 1])
        B[:, i] = inside
    for d in range(1, p + 1):
        m = len(knots) - 1 - d
        Bn = np.zeros((x.size, m), dtype=B.dtype)
        for l in range(m):
            den1 = knots[l + d] - knots[l]
            den2 = knots[l + d + 1] - knots[l + 1]
            if den1 > 0.0:
                Bn[:, l] += (x - knots[l]) / den1 * B[:, l]
            if den2 > 0.0:
                Bn[:, l] += (knots[l + d + 1] - x) / den2 * B[:, l + 1]
        B = Bn
    return B


def basis_derivative(knots, p, x):
    """First derivatives of all b_l^p at x, shape (len(x), k).

    Standard derivative formula of the recursion:
    (b_l^p)' = p/(xi_{l+p}-xi_l) b_l^{p-1} - p/(xi_{l+p+1}-xi_{l+1}) b_{l+1}^{p-1}."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if p == 0:
        return np.zeros((x.size, n_basis(knots, 0)))
    Bl = basis(knots, p - 1, x)
    k = n_basis(knots, p)
    D = np.zeros((x.size, k))
    for l in range(k):
        den1 = knots[l + p] - knots[l]
        den2 = knots[l + p + 1] - knots[l + 1]
        if den1 > 0.0:
            D[:, l] += p / den1 * Bl[:, l]
        if den2 > 0.0:
            D[:, l] -= p / den2 * Bl[:, l + 1]
    return D


def greville(knots, p):
    """Greville abscissae (xi_{l+1} + ... + xi_{l+p}) / p (for p = 0 the span midpoints)."""
    k = n_basis(knots, p)
    if p == 0:
        return np.array([(knots[l] + knots[l + 1]) / 2 for l in range(k)])
    return np.array([np.sum(knots[l + 1:l + p + 1]) / p for l in range(k)])


def refinement_matrix(p, j):
    """Knot-insertion matrix P with B_{j+1}(x) P = B_j(x) for all x (Sec. 2.3, nested spaces).

    S_p(Xi_{j,p}) is contained in S_p(Xi_{j+1,p}); the coarse basis is expanded in
    the fine basis by collocation at the fine Greville abscissae, where the fine
    collocation matrix is non-singular (Schoenberg-Whitney).  Shape (2^{j+1}+p, 2^j+p)."""
    kc = dyadic_knots(p, j)
    kf = dyadic_knots(p, j + 1)
    g = greville(kf, p)
    Bf = basis(kf, p, g)
    Bc = basis(kc, p, g)
    return np.linalg.solve(Bf, Bc)
