"""Pins of the oracle's surface maps, derivatives and point inversion."""
import numpy as np
import pytest

from oracle import assembly, geometry


@pytest.mark.parametrize("perturbed", [False, True])
def test_complex_step_matches_central_differences(perturbed):
    rng = np.random.default_rng(0)
    s, t = rng.uniform(0.05, 0.95, 20), rng.uniform(0.05, 0.95, 20)
    h = 1e-6
    for m in range(6):
        ds, dt = geometry.jacobian(m, s, t, perturbed)
        fs = (geometry.patch_map(m, s + h, t, perturbed) - geometry.patch_map(m, s - h, t, perturbed)) / (2 * h)
        ft = (geometry.patch_map(m, s, t + h, perturbed) - geometry.patch_map(m, s, t - h, perturbed)) / (2 * h)
        assert np.allclose(ds, fs, atol=1e-8)
        assert np.allclose(dt, ft, atol=1e-8)


def test_points_on_unit_sphere_and_outward():
    rng = np.random.default_rng(1)
    s, t = rng.uniform(0, 1, 30), rng.uniform(0, 1, 30)
    for m in range(6):
        X = geometry.patch_map(m, s, t)
        assert np.allclose(np.linalg.norm(X, axis=1), 1.0, atol=1e-15)
        ds, dt = geometry.jacobian(m, s, t)
        assert np.all(np.sum(np.cross(ds, dt) * X, axis=1) > 0)


@pytest.mark.parametrize("perturbed", [False, True])
def test_shared_edges_conform(perturbed):
    """Neighbouring maps agree on interfaces up to a rotation (Sec. 2.2): every edge point of a
    patch is a point of exactly one other patch's edge."""
    g = np.linspace(0, 1, 9)
    edges = []
    for m in range(6):
        for (s, t) in [(g, 0 * g), (g, 0 * g + 1), (0 * g, g), (0 * g + 1, g)]:
            edges.append(geometry.patch_map(m, s, t, perturbed))
    allpts = np.concatenate(edges)
    for e in edges:
        for x in e:
            hits = np.sum(np.linalg.norm(allpts - x, axis=1) < 1e-12)
            assert hits in (2, 6)  # edge interior: 2 copies; cube corner: 3 patches x 2 edges


def test_inversion_round_trip():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((500, 3))
    P = g / np.linalg.norm(g, axis=1, keepdims=True)
    patch, s, t = geometry.invert(P)
    assert np.all((s >= 0) & (s <= 1) & (t >= 0) & (t <= 1))
    for i in range(len(P)):
        assert np.allclose(geometry.patch_map(patch[i], s[i], t[i]), P[i], atol=1e-14)


def test_surface_area_of_unit_sphere():
    d = assembly.Discretisation(3, 3)
    one = np.ones(d.N)
    assert one @ (d.M @ one) == pytest.approx(4 * np.pi, rel=1e-7)
