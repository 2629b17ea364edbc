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
