"""White-noise load b ~ N(0, M) (oracle, test infrastructure only).

Sec. 3.3: the discrete load of white noise is normally distributed with
covariance M.  The paper draws it as sqrt(M) y; the load used for parity is the
element-wise factorisation b = sum_e R_e^T L_e z_e with M_e = L_e L_e^T (lower
Cholesky factor of the element mass matrix) and z_e ~ N(0, I) independent per
element.  Its covariance is sum_e R_e^T M_e R_e = M exactly, so b = L z with the
tall factor L = [R_1^T L_1, R_2^T L_2, ...] and M = L L^T.

Layout of z (one sample): elements in the order patch, ey, ex (ex fastest), each
with (p+1)^2 entries in element-local order (b, a), a (along s) fastest.
"""
import numpy as np


def element_factors(disc):
    """Lower Cholesky factors L_e of all element mass matrices, shape (n_el_total, nloc, nloc)."""
    return np.linalg.cholesky(disc.el_M)


def load(disc, z):
    """b = sum_e R_e^T L_e z_e for z of shape (nsamp, n_el_total * (p+1)^2)."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    L = element_factors(disc)
    nel, nloc = disc.el_dofs.shape
    out = np.zeros((z.shape[0], disc.N))
    for s in range(z.shape[0]):
        ze = z[s].reshape(nel, nloc)
        contrib = np.einsum("eij,ej->ei", L, ze)
        np.add.at(out[s], disc.el_dofs.reshape(-1), contrib.reshape(-1))
    return out


def factor_matrix(disc):
    """The tall factor L (N x n_el_total*(p+1)^2) with L L^T = M, for tiny meshes."""
    L = element_factors(disc)
    nel, nloc = disc.el_dofs.shape
    F = np.zeros((disc.N, nel * nloc))
    for e in range(nel):
        for i in range(nloc):
            F[disc.el_dofs[e, i], e * nloc:(e + 1) * nloc] += L[e, i, :]
    return F
