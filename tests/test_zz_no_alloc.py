"""The allocation-free operator apply (gf_space_apply_noalloc) against gf_space_apply, through the C ABI:
two calls in a row on one space, the second with fewer vectors (the shared work space keeps the first
call's contents), both operator kinds; and the size limit of the work space."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2605_24882_amd import gfield as g  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context(0)


@pytest.mark.parametrize("p,j,pert", [(2, 4, False), (3, 3, True)])
@pytest.mark.parametrize("kind", [g.GF_APPLY_STENCIL, g.GF_APPLY_SUMFACT])
def test_noalloc_apply_matches_apply(ctx, p, j, pert, kind):
    sp = g.Space(ctx, g.Geometry(ctx, pert), p, j)
    rng = np.random.default_rng(21)
    for nvec, sigma, ss in [(70, 16.3, 1.0), (5, 0.7, 2.5)]:
        x = torch.from_numpy(rng.standard_normal((nvec, sp.ndofs))).cuda()
        ref = sp.apply(sigma, ss, x, kind)
        y = torch.full_like(x, float("nan"))
        sp.apply_noalloc(sigma, ss, x, y, kind)
        torch.cuda.synchronize()
        scale = float(ref.abs().max())
        assert float((y - ref).abs().max()) <= 1e-13 * scale, (nvec, kind)


def test_noalloc_rejects_too_many_vectors(ctx):
    sp = g.Space(ctx, g.Geometry(ctx, False), 3, 7)  # 6 x 137^2 padded rows: 400 vectors exceed 256 MiB
    x = torch.zeros((400, sp.ndofs), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    st = g._lib.gf_space_apply_noalloc(sp.h, 1.0, 1.0, 400, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), g.GF_APPLY_STENCIL)
    assert st == g.GF_EINVAL
    assert b"work space" in g._lib.gf_last_error()
