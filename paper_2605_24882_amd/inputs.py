"""Seeded synthetic inputs shared by the GPU path's callers and by the oracle's tests.

This module holds random-number generation only, none of the method's
arithmetic: standard normal vectors for the element-wise white-noise factor,
uniform random points on the unit sphere and Gaussian targets.  Each caller
turns these into loads, losses and fields with its own code.
"""
import numpy as np


def noise_vectors(seeds, length):
    """One standard normal vector z of `length` entries per seed (float64), shape (len(seeds), length).

    Seed s draws its vector from numpy.random.default_rng(s)."""
    return np.stack([np.random.default_rng(s).standard_normal(length) for s in seeds])


def sphere_points_and_targets(npts, seed=7):
    """npts points uniform on the unit sphere (normalised 3D standard normals), then npts
    standard normal targets, both from numpy.random.default_rng(seed) in that order."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((npts, 3))
    pts = g / np.linalg.norm(g, axis=1, keepdims=True)
    y = rng.standard_normal(npts)
    return pts, y


def noise_length(p, level, npatch=6):
    """Entries of one element-wise noise vector: one (p+1)^2 block per element."""
    return npatch * (4 ** level) * (p + 1) ** 2


def torus_patches(R=2.0, r=1.0):
    """A torus with major radius R and minor radius r as 4 x 4 biquadratic rational Bezier patches
    (a synthetic stand-in for a multi-patch CAD surface: every corner joins four patches).

    The torus is the surface of revolution of the circle (R + r cos phi, r sin phi) about the z
    axis; both circles are split into quarters, each the rational quadratic arc with control points
    (cos a0, sin a0), (cos a0 + cos a1, sin a0 + sin a1), (cos a1, sin a1) and weights 1, 1/sqrt(2),
    1 (a1 = a0 + pi/2).  Patch 4 i + k covers the quarter i of the revolution (along s) and the
    quarter k of the profile circle (along t); neighbouring patches share their edge control points.

    Returns (deg_u, deg_v, ncoef [16][2], knots (flat: per patch s then t), ctrl [16][3][3][4])
    in the layout of gf_geometry_nurbs."""
    h = 1.0 / np.sqrt(2.0)

    def quarter(i):
        a0, a1 = i * np.pi / 2.0, (i + 1) * np.pi / 2.0
        c0, s0, c1, s1 = np.cos(a0), np.sin(a0), np.cos(a1), np.sin(a1)
        # exact values at multiples of pi/2 (cos and sin of them are 0 or +-1)
        c0, s0, c1, s1 = (float(np.rint(v)) for v in (c0, s0, c1, s1))
        return [(c0, s0, 1.0), (c0 + c1, s0 + s1, h), (c1, s1, 1.0)]

    knots1 = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    ncoef, knots, ctrl = [], [], []
    for i in range(4):
        rev = quarter(i)
        for k in range(4):
            prof = quarter(k)
            net = np.empty((3, 3, 4))
            for b, (pc, ps, pw) in enumerate(prof):  # along t: the profile circle
                rho, z = R + r * pc, r * ps  # profile control point in the (rho, z) half-plane
                for a, (qc, qs, qw) in enumerate(rev):  # along s: the revolution
                    net[b, a] = (rho * qc, rho * qs, z, pw * qw)
            ncoef.append((3, 3))
            knots.extend(knots1 + knots1)
            ctrl.append(net)
    return 2, 2, np.array(ncoef, dtype=np.int32), np.array(knots), np.array(ctrl)
