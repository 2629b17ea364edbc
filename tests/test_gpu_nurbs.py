"""GPU parity on a NURBS multi-patch surface: the 4 x 4 patch torus (R = 2, r = 1, biquadratic
rational Bezier patches, four patches at every corner) through gf_geometry_nurbs, against the
oracle's own NURBS evaluation (complex-step metric, Greville-point gluing).

Tolerances as the sphere parity tests: operator and load 1e-13 relative, FP64 fields 1e-10 in
the M-norm at CG rtol 1e-13, mixed precision 1e-10 with the same FP64 outer residual; at a size
the oracle does not solve in a test, the constant-load closed form (1e-9, rtol 1e-12).
"""
import math

import numpy as np
import pytest

from oracle import assembly, evaluate, fractional, geometry, noise, sinc
from paper_2605_24882_amd import inputs

pytestmark = pytest.mark.gpu

g = pytest.importorskip("paper_2605_24882_amd.gfield")

R, RR = 2.0, 1.0
NP = 16


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return g.Context(0)


@pytest.fixture(scope="module")
def geo(ctx):
    return g.Geometry.nurbs(ctx, *inputs.torus_patches(R, RR))


_surf = geometry.NurbsSurface(*inputs.torus_patches(R, RR))
_spaces, _discs = {}, {}


def space(ctx, geo, p, j):
    if (p, j) not in _spaces:
        _spaces[(p, j)] = g.Space(ctx, geo, p, j)
    return _spaces[(p, j)]


def disc(p, j):
    if (p, j) not in _discs:
        _discs[(p, j)] = assembly.Discretisation(p, j, _surf)
    return _discs[(p, j)]


def mrel(d, u, ref):
    out = 0.0
    for a, b in zip(np.atleast_2d(u), np.atleast_2d(ref)):
        e = a - b
        out = max(out, math.sqrt(e @ (d.M @ e)) / math.sqrt(b @ (d.M @ b)))
    return out


CASES = [(2, 2), (3, 2), (1, 3), (2, 3)]


@pytest.mark.parametrize("p,j", CASES)
def test_torus_dofmap_matches_oracle(ctx, geo, p, j):
    sp, d = space(ctx, geo, p, j), disc(p, j)
    n = 2 ** j + p
    assert geo.npatch == NP
    assert sp.ndofs == d.N == NP * (n - 1) ** 2
    assert np.array_equal(sp.dofmap(), d.l2g)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p,j", CASES)
def test_torus_apply_matches_oracle(ctx, geo, p, j, kind):
    sp, d = space(ctx, geo, p, j), disc(p, j)
    x = np.random.default_rng(11).standard_normal((3, d.N))
    for sigma, ss in [(1.0, 0.0), (0.0, 1.0), (9.3, 1.0)]:
        y = sp.apply(sigma, ss, x, kind)
        ref = np.stack([(sigma * d.M + ss * d.S) @ v for v in x])
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), (sigma, ss)


@pytest.mark.parametrize("p,j", [(2, 2), (3, 2)])
def test_torus_white_noise_matches_oracle(ctx, geo, p, j):
    sp, d = space(ctx, geo, p, j), disc(p, j)
    assert sp.noise_length == inputs.noise_length(p, j, NP)
    z = inputs.noise_vectors([0, 1, 2], sp.noise_length)
    b = sp.white_noise(z)
    ref = noise.load(d, z)
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("beta", [0.7, 1.6])
@pytest.mark.parametrize("prec", [0, 1])
def test_torus_sample_matches_oracle(ctx, geo, beta, prec):
    sp, d = space(ctx, geo, 2, 3), disc(2, 3)
    z = inputs.noise_vectors([4, 5], sp.noise_length)
    b = noise.load(d, z)
    u, st = sp.sample(3.0, beta, b, h=0.4, k_minus=12, k_plus=12, precision=prec, rtol=1e-13)
    ref = fractional.sample(d.M, d.S, 3.0, beta, 0.4, 12, 12, b)
    err = mrel(d, u, ref)
    print(f"torus p=2 j=3 beta={beta} prec={prec}: rel. M-norm error {err:.2e}, iterations {st['max_iters']}")
    assert err <= 1e-10
    # multigrid on a surface with four patches at every corner: measured 7-8 iterations
    assert st["max_iters"] <= 10, st["max_iters"]


def test_torus_eval_matches_oracle(ctx, geo):
    sp, d = space(ctx, geo, 3, 2), disc(3, 2)
    rng = np.random.default_rng(8)
    patch = rng.integers(0, NP, 50).astype(np.int32)
    st = rng.random((50, 2))
    u = rng.standard_normal((2, d.N))
    vals = sp.eval(patch, st, u)
    ref = (evaluate.phi_matrix(d, patch, st[:, 0], st[:, 1]) @ u.T).T
    assert np.abs(vals - ref).max() <= 1e-13 * np.abs(ref).max()


def test_torus_constant_load_closed_form_at_size(ctx, geo):
    """p = 2, 64 x 64 elements per patch (16 patches, 67,600 unknowns): u = kappa^-2n Q(kappa^2) 1."""
    import torch
    sp = space(ctx, geo, 2, 6)
    assert sp.ndofs == NP * 65 ** 2
    one = torch.ones(1, sp.ndofs, dtype=torch.float64, device="cuda")
    b = sp.apply(1.0, 0.0, one)
    area = b.sum().item()
    assert abs(area - 4 * math.pi ** 2 * R * RR) <= 1e-12 * area
    kappa, beta = 10.0, 1.6
    u, st = sp.sample(kappa, beta, b, h=0.4, k_minus=20, k_plus=20, precision=1, rtol=1e-12, max_iter=2000)
    n, bf = fractional.split_plain(beta)
    expect = kappa ** (-2 * n) * sinc.sinc_sum(kappa ** 2, bf, 0.4, 20, 20)
    print(f"torus 67,600 unknowns: constant load, max abs dev {(u - expect).abs().max().item():.2e}, "
          f"iterations {st['max_iters']}")
    assert (u - expect).abs().max().item() <= 1e-9 * abs(expect)


# ---- open surfaces (unmatched edges: natural boundary condition)
from tests import open_surfaces  # noqa: E402

_open = {}


def open_case(ctx, name, p, j):
    key = (name, p, j)
    if key not in _open:
        args = getattr(open_surfaces, name)()
        geo_ = g.Geometry.nurbs(ctx, *args)
        _open[key] = (g.Space(ctx, geo_, p, j), assembly.Discretisation(p, j, geometry.NurbsSurface(*args)))
    return _open[key]


@pytest.mark.parametrize("name,p,j", [("square", 2, 3), ("strip", 2, 3), ("strip", 3, 2)])
def test_open_surface_parity(ctx, name, p, j):
    """Dofmap, both operator kinds and FP64 / mixed fields against the oracle on open patches: the
    rows of boundary unknowns with a single copy run the full epilogue."""
    sp, d = open_case(ctx, name, p, j)
    assert np.array_equal(sp.dofmap(), d.l2g)
    x = np.random.default_rng(4).standard_normal((2, d.N))
    for kind in (0, 1):
        y = sp.apply(7.0, 1.0, x, kind)
        ref = np.stack([(7.0 * d.M + d.S) @ v for v in x])
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    z = inputs.noise_vectors([1, 2], sp.noise_length)
    b = noise.load(d, z)
    assert np.abs(sp.white_noise(z) - b).max() <= 1e-13 * np.abs(b).max()
    ref = fractional.sample(d.M, d.S, 2.0, 1.3, 0.4, 10, 10, b)
    for prec in (0, 1):
        u, st = sp.sample(2.0, 1.3, b, h=0.4, k_minus=10, k_plus=10, precision=prec, rtol=1e-13)
        assert mrel(d, u, ref) <= 1e-10, prec


@pytest.mark.parametrize("p,j,lc", [(3, 2, -1), (2, 3, 1)])
def test_torus_large_coarse_level(ctx, geo, p, j, lc):
    """Coarsest levels whose right-hand sides do not fit the LDS of the coarse solve (144 unknowns on
    the 16-patch torus: degree 3 at level 0, degree 2 at level 1) read them from memory."""
    sp = g.Space(ctx, geo, p, j, mg_levels=0 if lc < 0 else j - lc + 1)
    d = disc(p, j)
    b = noise.load(d, inputs.noise_vectors([9], sp.noise_length))
    ref = fractional.sample(d.M, d.S, 3.0, 1.6, 0.4, 10, 10, b)
    for prec in (0, 1):
        u, st = sp.sample(3.0, 1.6, b, h=0.4, k_minus=10, k_plus=10, precision=prec, rtol=1e-13)
        assert mrel(d, u, ref) <= 1e-10, prec


def test_torus_improved_split_bpx_sqrt_mass_and_gradient(ctx, geo):
    """The rows built on the solver, on the NURBS torus (p = 2, 4 x 4 elements per patch): the
    improved split, the BPX preconditioner, the sqrt(M) load and d loss / d kappa, each against the
    oracle."""
    import scipy.sparse as sps
    from oracle import gradient, sqrt_mass
    sp, d = space(ctx, geo, 2, 2), disc(2, 2)
    b = noise.load(d, inputs.noise_vectors([3, 4], sp.noise_length))
    # improved split: beta = 2.3 -> 1 integer solve + the rule for 0.65 twice
    u, _ = sp.sample(3.0, 2.3, b, h=0.4, k_minus=10, k_plus=10, rtol=1e-13, split=g.GF_SPLIT_IMPROVED)
    ref = fractional.sample(d.M, d.S, 3.0, 2.3, 0.4, 10, 10, b, mode="improved")
    assert mrel(d, u, ref) <= 1e-10
    # BPX, both precisions
    ref = fractional.sample(d.M, d.S, 3.0, 1.6, 0.4, 10, 10, b)
    for prec in (0, 1):
        u, _ = sp.sample(3.0, 1.6, b, h=0.4, k_minus=10, k_plus=10, precision=prec, rtol=1e-13, max_iter=3000,
                         preconditioner=g.GF_PRECOND_BPX)
        assert mrel(d, u, ref) <= 1e-10, prec
    # sqrt(M) y with the oracle's bounds
    lo, hi = sqrt_mass.dense_bounds(d.M)
    lo, hi = 0.99 * lo, 1.01 * hi
    y = np.random.default_rng(21).standard_normal((2, d.N))
    f, _ = sp.sqrt_mass(y, khat=12, lo=lo, hi=hi, rtol=1e-13)
    fr = sqrt_mass.apply(d.M, y, 12, lo, hi)
    assert np.abs(f - fr).max() <= 1e-10 * np.abs(fr).max()
    # d loss / d kappa at 40 parameter points
    rng = np.random.default_rng(22)
    patch = rng.integers(0, NP, 40).astype(np.int32)
    st = rng.random((40, 2))
    yt = rng.standard_normal(40)
    Phi = sps.csr_matrix(evaluate.phi_matrix(d, patch, st[:, 0], st[:, 1]))
    kw = dict(h=0.4, k_minus=10, k_plus=10, rtol=1e-13)
    u, tape, _ = sp.sample_tape(3.0, 1.6, b, **kw)
    grad, _ = tape.grad_kappa(sp.eval_adjoint(patch, st, sp.eval(patch, st, u) - yt[None, :]))
    tape.close()
    gref, _ = gradient.adjoint(d.M, d.S, 3.0, 1.6, 0.4, 10, 10, b, Phi, yt)
    assert np.abs(grad - gref).max() <= 1e-9 * np.abs(gref).max()


def test_torus_workload_subset_matches_oracle(ctx, geo):
    """The torus workload of bench.py at full size (p = 2, 32 x 32 elements per 16 patches, 17,424
    unknowns, kappa = 10, beta = 1.6, 41 nodes): samples 0 and 1 of the 64 against the oracle."""
    sp, d = space(ctx, geo, 2, 5), disc(2, 5)
    assert sp.ndofs == 17424
    b = noise.load(d, inputs.noise_vectors([0, 1], sp.noise_length))
    u, st = sp.sample(10.0, 1.6, b, h=0.4, k_minus=20, k_plus=20, rtol=1e-12)
    ref = fractional.sample(d.M, d.S, 10.0, 1.6, 0.4, 20, 20, b)
    assert mrel(d, u, ref) <= 1e-10
    assert st["max_iters"] <= 9, st["max_iters"]  # measured 7
