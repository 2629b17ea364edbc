"""Square root of the mass matrix applied to a vector (oracle, test infrastructure only).

Sec. 3.3, eq. (sqrt): with bounds 0 < m < lambda_min(M), Mu > lambda_max(M) and the parameter
q = 1 - m/Mu,
    sqrt(M) y ~ (2 K sqrt(m) / (pi Khat)) M sum_{k=1..Khat} dn(t_k|q)/cn(t_k|q)^2 (M + w_k^2 I)^-1 y,
    w_k = sqrt(m) sn(t_k|q)/cn(t_k|q),   t_k = (k - 1/2) K / Khat,
with sn, cn, dn the Jacobi elliptic functions of parameter q.  Reading of the garbled constant: the
paper prints E (the complete integral of the second kind); the rule is the midpoint rule on
[0, K] after the substitution w = sqrt(m) sn/cn, so both the prefactor and the nodes use K(q), the
complete elliptic integral of the first kind at the same parameter as sn, cn, dn.

Each (M + w_k^2 I) solve is a sparse LU; the sum runs over k in ascending order.
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import ellipj, ellipk


def rule(m, Mu, khat):
    """(w2, a, c): shifts w_k^2, weights dn/cn^2 and the prefactor 2 K sqrt(m)/(pi Khat)."""
    q = 1.0 - m / Mu
    K = ellipk(q)
    t = (np.arange(1, khat + 1) - 0.5) * K / khat
    sn, cn, dn, _ = ellipj(t, q)
    return m * (sn / cn) ** 2, dn / cn ** 2, 2.0 * K * math.sqrt(m) / (math.pi * khat)


def scalar(lam, m, Mu, khat):
    """The rule applied to a scalar lam (an eigenvalue of M): approximates sqrt(lam)."""
    w2, a, c = rule(m, Mu, khat)
    lam = np.asarray(lam, dtype=np.float64)
    return c * lam * np.sum(a[:, None] / (lam.reshape(1, -1) + w2[:, None]), axis=0).reshape(lam.shape)


def apply(M, y, khat, m, Mu):
    """sqrt(M) y for y of shape (nsamp, N) by the rule; returns shape (nsamp, N)."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    w2, a, c = rule(m, Mu, khat)
    N = M.shape[0]
    acc = np.zeros_like(y)
    for k in range(khat):  # ascending k
        lu = spla.splu((M + w2[k] * sp.identity(N, format="csc")).tocsc())
        acc = acc + a[k] * np.stack([lu.solve(v) for v in y])
    return c * np.stack([M @ v for v in acc])


def dense_bounds(M):
    """Extreme eigenvalues of M (dense, tiny meshes)."""
    ev = sla.eigvalsh(M.toarray())
    return ev[0], ev[-1]
