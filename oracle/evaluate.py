"""Point evaluation of a spline field on the surface (oracle, test infrastructure only).

A function of S^0_{j,p} restricted to patch m is the pull-back of the tensor
spline sum c[m, iy, ix] b_ix(s) b_iy(t) (Sec. 2.3); its value at the surface
point F_m(s, t) is that sum.  Phi maps global coefficients to point values.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline


def phi_matrix(disc, patch, s, t):
    """Sparse (npts x N) matrix of basis values at points given by patch index and (s, t)."""
    rows, cols, vals = [], [], []
    for i in range(len(patch)):
        bx = bspline.basis(disc.knots, disc.p, [s[i]])[0]
        by = bspline.basis(disc.knots, disc.p, [t[i]])[0]
        for iy in np.nonzero(by)[0]:
            for ix in np.nonzero(bx)[0]:
                rows.append(i)
                cols.append(disc.l2g[patch[i], iy, ix])
                vals.append(by[iy] * bx[ix])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(patch), disc.N))
