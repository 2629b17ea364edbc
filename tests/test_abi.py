"""Host-side checks of the C ABI: the library loads, exports every declared entry point,
validates arguments before touching a device, and its host-only calls match the oracle."""
import os
import re

import numpy as np
import pytest

from paper_2605_24882_amd import gfield as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gfield.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(g._lib, n), n
        assert n in g.EXPORTED, n


def test_abi_version():
    assert g.abi_version() == 2


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_context_without_device_is_edevice():
    with pytest.raises(g.GfieldError) as e:
        g.Context(0, use_torch_stream=False)
    assert e.value.status == g.GF_EDEVICE


def test_null_handles_are_einval():
    import ctypes
    x = np.zeros(4)
    assert g._lib.gf_space_apply(None, 1.0, 1.0, 1, x.ctypes.data, x.ctypes.data, g.GF_HOST, 0) == g.GF_EINVAL
    assert b"null" in g._lib.gf_last_error()
    out = ctypes.c_void_p()
    assert g._lib.gf_space_create(None, None, 2, 2, 0, 0, ctypes.byref(out)) == g.GF_EINVAL
    for amp in (1.0, -1.5, float("nan"), float("inf")):
        assert g._lib.gf_geometry_cubesphere(None, amp, ctypes.byref(out)) == g.GF_EINVAL
    rule = g.QuadRule(0.4, 15, 15)
    opts = g.SolveOpts(0, 1e-10, 100, 0, 0, 0)
    st = g.SolveStats()
    assert g._lib.gf_sample(None, 4.0, 0.75, ctypes.byref(rule), ctypes.byref(opts), 1, x.ctypes.data,
                            x.ctypes.data, g.GF_HOST, ctypes.byref(st)) == g.GF_EINVAL
    items = (g.BatchItem * 1)()
    assert g._lib.gf_sample_batch(None, 1, items, ctypes.byref(opts), g.GF_HOST, ctypes.byref(st)) == g.GF_EINVAL
    rate = ctypes.c_double(0.0)
    assert g._lib.gf_probe_fma(None, g.GF_PREC_FP64, ctypes.byref(rate)) == g.GF_EINVAL


def test_locate_matches_oracle_inversion():
    from oracle import geometry
    from paper_2605_24882_amd import inputs
    pts, _ = inputs.sphere_points_and_targets(1000, seed=7)
    geo = g.Geometry(None, perturb_amp=0.0)
    patch, st = geo.locate(pts)
    op, os_, ot = geometry.invert(pts)
    assert np.array_equal(patch, op)
    assert np.allclose(st[:, 0], os_, atol=1e-15) and np.allclose(st[:, 1], ot, atol=1e-15)
    with pytest.raises(g.GfieldError):
        geo.locate(np.zeros((1, 3)))


def test_sqrt_mass_rule_matches_oracle():
    """The library's Jacobi elliptic functions (arithmetic-geometric mean) against SciPy's, through the
    nodes and weights of the square-root rule; host computation, no device needed."""
    from oracle import sqrt_mass
    for lo, hi, khat in [(0.1, 1.0, 8), (1e-4, 3e-3, 16), (0.02, 50.0, 24), (0.5, 0.5000001, 3)]:
        w2, a, c = g.sqrt_mass_rule(lo, hi, khat)
        rw2, ra, rc = sqrt_mass.rule(lo, hi, khat)
        assert np.allclose(w2, rw2, rtol=1e-12, atol=0) and np.allclose(a, ra, rtol=1e-12) and abs(c - rc) <= 1e-13 * rc
    import ctypes
    x = np.zeros(4)
    cc = ctypes.c_double()
    assert g._lib.gf_sqrt_mass_rule(1.0, 0.5, 4, x.ctypes.data, x.ctypes.data, ctypes.byref(cc)) == g.GF_EINVAL


def test_nurbs_geometry_accepts_the_torus_and_validates_input():
    """gf_geometry_nurbs on the host: the 4 x 4 patch torus is accepted (its interfaces glue), and
    malformed nets are refused before any device work."""
    from paper_2605_24882_amd import inputs
    du, dv, nc, kn, cp = inputs.torus_patches(2.0, 1.0)
    geo = g.Geometry.nurbs(None, du, dv, nc, kn, cp)
    assert geo.npatch == 16
    geo.close()

    def status(du_, dv_, nc_, kn_, cp_):
        with pytest.raises(g.GfieldError) as e:
            g.Geometry.nurbs(None, du_, dv_, nc_, kn_, cp_)
        return e.value.status

    bad = cp.copy()
    bad[3, 1, 1, 3] = 0.0  # a zero weight
    assert status(du, dv, nc, kn, bad) == g.GF_EINVAL
    bad_k = kn.copy()
    bad_k[0] = -0.5  # not open on [0, 1]
    assert status(du, dv, nc, bad_k, cp) == g.GF_EINVAL
    assert status(5, dv, nc, kn, cp) == g.GF_EINVAL  # degree out of range
    # three patches on one edge: patch 0 twice
    assert status(du, dv, np.concatenate([nc, nc[:1]]), np.concatenate([kn, kn[:12]]),
                  np.concatenate([cp, cp[:1]])) == g.GF_EINVAL
    # an edge collapsed to a point
    deg = cp.copy()
    deg[0, 0, :, :3] = deg[0, 0, 0, :3]
    assert status(du, dv, nc, kn, deg) == g.GF_EUNSUPPORTED


def test_nurbs_locate_recovers_parameters():
    """gf_locate on the NURBS torus (host work only): points made by the oracle's map from random
    (patch, s, t) are found again -- the same patch and parameters away from patch edges, and a
    parameter pair whose image is the point everywhere -- and a point off the surface goes to its
    closest point."""
    from oracle import geometry
    from paper_2605_24882_amd import inputs
    args = inputs.torus_patches(2.0, 1.0)
    surf = geometry.NurbsSurface(*args)
    geo = g.Geometry.nurbs(None, *args)
    rng = np.random.default_rng(31)
    m = rng.integers(0, 16, 200)
    st = rng.uniform(0.02, 0.98, (200, 2))
    pts = np.stack([geometry.patch_map(int(mi), s[0], s[1], surf) for mi, s in zip(m, st)])
    patch, st2 = geo.locate(pts)
    assert np.array_equal(patch, m)
    assert np.abs(st2 - st).max() <= 1e-10
    # corners and edges: any (patch, s, t) whose image is the point
    edge = np.array([[0.0, 0.0], [1.0, 0.5], [0.5, 1.0], [1.0, 1.0]])
    pts = np.stack([geometry.patch_map(5, s[0], s[1], surf) for s in edge])
    patch, st2 = geo.locate(pts)
    back = np.stack([geometry.patch_map(int(pi), s[0], s[1], surf) for pi, s in zip(patch, st2)])
    assert np.abs(back - pts).max() <= 1e-12
    # off the surface: (3.5, 0, 0) is 0.5 outside the outer equator
    patch, st2 = geo.locate(np.array([[3.5, 0.0, 0.0]]))
    x = geometry.patch_map(int(patch[0]), st2[0, 0], st2[0, 1], surf)
    assert np.abs(x - np.array([3.0, 0.0, 0.0])).max() <= 1e-10
