"""Open NURBS surfaces for tests (plain data): the unit square as one bilinear patch, and the strip
[0, 2] x [0, 1] as two patches whose s axes run towards the shared edge x = 1 from both sides
(the edge is s = 1 on both patches).  Their unmatched edges are boundaries with the natural
condition, so S is the Neumann Laplacian with eigenvalues pi^2 (m^2 / Lx^2 + n^2)."""
import numpy as np

KNOTS1 = [0.0, 0.0, 1.0, 1.0]


def square():
    ctrl = np.array([[[0.0, 0.0, 0.0, 1.0], [1.0, 0.0, 0.0, 1.0]],
                     [[0.0, 1.0, 0.0, 1.0], [1.0, 1.0, 0.0, 1.0]]])
    return 1, 1, np.array([[2, 2]], dtype=np.int32), np.array(KNOTS1 * 2), ctrl[None]


def strip():
    left = np.array([[[0.0, 0.0, 0.0, 1.0], [1.0, 0.0, 0.0, 1.0]],
                     [[0.0, 1.0, 0.0, 1.0], [1.0, 1.0, 0.0, 1.0]]])
    right = np.array([[[2.0, 0.0, 0.0, 1.0], [1.0, 0.0, 0.0, 1.0]],
                      [[2.0, 1.0, 0.0, 1.0], [1.0, 1.0, 0.0, 1.0]]])
    return 1, 1, np.array([[2, 2], [2, 2]], dtype=np.int32), np.array(KNOTS1 * 4), np.stack([left, right])


def neumann_eigenvalues(lx, count):
    """The smallest `count` eigenvalues pi^2 (m^2 / lx^2 + n^2), m, n >= 0, of the rectangle."""
    vals = sorted(np.pi ** 2 * (m * m / lx ** 2 + n * n) for m in range(12) for n in range(12))
    return np.array(vals[:count])
