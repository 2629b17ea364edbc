"""Surfaces: six-patch sphere, perturbed sphere, NURBS patches (oracle, test infrastructure only).

Sec. 2.2 asks for patch maps F_m: [0,1]^2 -> Gamma_m that agree on shared
interfaces up to a rotation of the reference square.  Sec. 4.1 uses the unit
sphere split into six patches; the paper's own map is only shown as a picture,
so the radial projection of the cube faces is used:

    a = 2s - 1, b = 2t - 1,
    patch 0 (+x): v = ( 1, a, b)     patch 1 (-x): v = (-1, b, a)
    patch 2 (+y): v = ( b, 1, a)     patch 3 (-y): v = ( a,-1, b)
    patch 4 (+z): v = ( a, b, 1)     patch 5 (-z): v = ( b, a,-1)
    F_m(s, t) = v / |v|,

each oriented so that dF/ds x dF/dt points outward.  The perturbed sphere
scales the unit-sphere point xh by r(xh) = 1 + amp sin(3x) sin(2y) cos(z) (amp = 0.15 for
the perturbed sphere of the workloads; `perturbed` may also be a number, the amplitude).

A NURBS surface (Sec. 2.2, definition of the geometry) is a list of rational
tensor-product B-spline patches F_m(s, t) = sum N_a(s) N_b(t) w_ab X_ab /
sum N_a(s) N_b(t) w_ab; `NurbsSurface` holds them, and every function below that
takes `perturbed` also accepts a NurbsSurface in its place.

Derivatives are taken by complex-step differentiation,
dF/ds = Im F(s + i eps, t) / eps with eps = 1e-30, exact to rounding for the
analytic maps used here (for NURBS, inside a knot span); no hand-derived
derivative formula is involved.
"""
import numpy as np

from . import bspline

NPATCH = 6
EPS_CS = 1e-30


class NurbsSurface:
    """Patches of degrees (du, dv); ncoef[m] = (control points along s, along t); knots flat, per
    patch the s then the t knot vector; ctrl[m] of shape (nt, ns, 4) = (x, y, z, weight)."""

    def __init__(self, du, dv, ncoef, knots, ctrl):
        self.du, self.dv = int(du), int(dv)
        self.npatch = len(ncoef)
        self.patches = []
        off = 0
        for m, (ns, nt) in enumerate(np.asarray(ncoef)):
            U = np.asarray(knots[off:off + ns + self.du + 1], dtype=np.float64)
            off += ns + self.du + 1
            V = np.asarray(knots[off:off + nt + self.dv + 1], dtype=np.float64)
            off += nt + self.dv + 1
            C = np.asarray(ctrl[m], dtype=np.float64).reshape(nt, ns, 4)
            self.patches.append((U, V, C))

    def point(self, m, s, t):
        """F_m(s, t) of shape s.shape + (3,); analytic in s and t (complex parameters allowed)."""
        U, V, C = self.patches[m]
        s = np.asarray(s)
        t = np.asarray(t)
        shape = np.broadcast(s, t).shape
        sf = np.broadcast_to(s, shape).reshape(-1)
        tf = np.broadcast_to(t, shape).reshape(-1)
        Bs = bspline.basis_analytic(U, self.du, sf)  # (npts, ns)
        Bt = bspline.basis_analytic(V, self.dv, tf)  # (npts, nt)
        w = C[..., 3]
        den = np.einsum("pb,pa,ba->p", Bt, Bs, w)
        num = np.einsum("pb,pa,bac->pc", Bt, Bs, C[..., :3] * w[..., None])
        return (num / den[:, None]).reshape(shape + (3,))


def npatch(surface):
    """Number of patches of the surface (`perturbed` flag or NurbsSurface)."""
    return surface.npatch if isinstance(surface, NurbsSurface) else NPATCH


def cube_point(m, s, t):
    """Unnormalised cube-face point v for patch m at parameters (s, t); works for complex input."""
    a = 2.0 * s - 1.0
    b = 2.0 * t - 1.0
    one = np.ones_like(a)
    if m == 0:
        return np.stack([one, a, b], axis=-1)
    if m == 1:
        return np.stack([-one, b, a], axis=-1)
    if m == 2:
        return np.stack([b, one, a], axis=-1)
    if m == 3:
        return np.stack([a, -one, b], axis=-1)
    if m == 4:
        return np.stack([a, b, one], axis=-1)
    if m == 5:
        return np.stack([b, a, -one], axis=-1)
    raise ValueError("patch index out of range")


def amplitude(perturbed):
    """Perturbation amplitude of the sphere family: False -> 0 (the unit sphere), True -> 0.15 (the
    perturbed sphere of the workloads), a number -> that amplitude."""
    if perturbed is True:
        return 0.15
    if perturbed is False or perturbed is None:
        return 0.0
    return float(perturbed)


def radius(xh, amp=0.15):
    """r(x, y, z) = 1 + amp sin(3x) sin(2y) cos(z) at the unit-sphere point xh."""
    return 1.0 + amp * np.sin(3.0 * xh[..., 0]) * np.sin(2.0 * xh[..., 1]) * np.cos(xh[..., 2])


def patch_map(m, s, t, perturbed=False):
    """F_m(s, t) in R^3 (analytic in s, t, so it accepts complex parameters)."""
    if isinstance(perturbed, NurbsSurface):
        return perturbed.point(m, s, t)
    s = np.asarray(s)
    t = np.asarray(t)
    v = cube_point(m, s, t)
    nrm = np.sqrt(np.sum(v * v, axis=-1))  # no conjugation: keeps the map analytic
    xh = v / nrm[..., None]
    amp = amplitude(perturbed)
    if amp != 0.0:
        return radius(xh, amp)[..., None] * xh
    return xh


def jacobian(m, s, t, perturbed=False):
    """(dF/ds, dF/dt), each of shape (..., 3), by complex-step differentiation."""
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    ds = np.imag(patch_map(m, s + 1j * EPS_CS, t + 0j, perturbed)) / EPS_CS
    dt = np.imag(patch_map(m, s + 0j, t + 1j * EPS_CS, perturbed)) / EPS_CS
    return ds, dt


def first_fundamental_form(m, s, t, perturbed=False):
    """K_m = J^T J and the surface measure a_m = sqrt(det K_m) (Sec. 3.2)."""
    ds, dt = jacobian(m, s, t, perturbed)
    k11 = np.sum(ds * ds, axis=-1)
    k12 = np.sum(ds * dt, axis=-1)
    k22 = np.sum(dt * dt, axis=-1)
    det = k11 * k22 - k12 * k12
    return k11, k12, k22, np.sqrt(det)


def invert(points):
    """Patch index and parameters (s, t) of surface points (radial inverse of the maps above).

    The direction xh = x/|x| decides: the coordinate of largest modulus picks the
    face, the two others divided by it give the cube-face coordinates (a, b)."""
    P = np.asarray(points, dtype=np.float64)
    xh = P / np.linalg.norm(P, axis=-1, keepdims=True)
    ax = np.argmax(np.abs(xh), axis=-1)
    patch = np.empty(len(P), dtype=np.int64)
    s = np.empty(len(P))
    t = np.empty(len(P))
    for i, (x, y, z) in enumerate(xh):
        c = ax[i]
        if c == 0:
            m = 0 if x > 0 else 1
            u, w = y / abs(x), z / abs(x)
            a, b = (u, w) if m == 0 else (w, u)
        elif c == 1:
            m = 2 if y > 0 else 3
            u, w = x / abs(y), z / abs(y)
            a, b = (w, u) if m == 2 else (u, w)
        else:
            m = 4 if z > 0 else 5
            u, w = x / abs(z), y / abs(z)
            a, b = (u, w) if m == 4 else (w, u)
        patch[i] = m
        s[i] = (a + 1.0) / 2.0
        t[i] = (b + 1.0) / 2.0
    return patch, s, t
