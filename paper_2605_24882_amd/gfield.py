"""ctypes binding of libgfield.so (the C ABI declared in include/gfield.h).

Argument marshalling only: every step of the computation runs in the HIP library.
Arrays are either NumPy arrays (host memory, GF_HOST) or torch tensors on the
context's GPU (device memory, GF_DEVICE); outputs are returned in the same kind
of container as the main input.  PyTorch supplies device memory and the stream.

If the library has not been built, importing this module raises ImportError --
there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

# torch first: the library then binds to the HIP runtime torch already loaded, so that one
# runtime serves both (two HIP/HSA runtimes in one process do not see the device)
try:
    import torch  # noqa: F401
except ImportError:  # host-only use (argument checks, gf_locate)
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfield.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_24882_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EDEVICE, GF_ENOCONV, GF_EBREAKDOWN, GF_EUNSUPPORTED = range(7)
GF_HOST, GF_DEVICE = 0, 1
GF_APPLY_STENCIL, GF_APPLY_SUMFACT = 0, 1
GF_PROLONG, GF_RESTRICT = 0, 1
GF_PREC_FP64, GF_PREC_MIXED = 0, 1
GF_FLAG_TIME_APPLY = 1
GF_FLAG_NO_GRAPH = 2
GF_FLAG_MASS_SHIFT = 4
GF_PRECOND_VCYCLE, GF_PRECOND_BPX = 0, 1
GF_SPLIT_PLAIN, GF_SPLIT_IMPROVED = 0, 1
STATUS_NAMES = {0: "GF_OK", 1: "GF_EINVAL", 2: "GF_ENOMEM", 3: "GF_EDEVICE", 4: "GF_ENOCONV",
                5: "GF_EBREAKDOWN", 6: "GF_EUNSUPPORTED"}


class QuadRule(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("k_minus", ctypes.c_int32), ("k_plus", ctypes.c_int32),
                ("split", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("apply_kind", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("preconditioner", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("n_systems", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("max_rel_resid", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("apply_ms", ctypes.c_double),
                ("apply_launches", ctypes.c_int32), ("apply_rows", ctypes.c_int32),
                ("apply_col_sum", ctypes.c_double), ("apply_bytes", ctypes.c_double),
                ("smooth_ms", ctypes.c_double), ("smooth_launches", ctypes.c_int32),
                ("smooth_bytes", ctypes.c_double), ("host_syncs", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [("space", ctypes.c_void_p), ("kappa", ctypes.c_double), ("beta", ctypes.c_double),
                ("rule", QuadRule), ("nsamp", ctypes.c_int32), ("b", ctypes.c_void_p), ("u", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_SIGS = {
    "gf_last_error": (ctypes.c_char_p, []),
    "gf_abi_version": (ctypes.c_int, []),
    "gf_context_create": (_i32, [_i32, _vp, ctypes.POINTER(_vp)]),
    "gf_context_destroy": (None, [_vp]),
    "gf_probe_fma": (_i32, [_vp, _i32, ctypes.POINTER(ctypes.c_double)]),
    "gf_geometry_cubesphere": (_i32, [_vp, _dbl, ctypes.POINTER(_vp)]),
    "gf_geometry_nurbs": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "gf_geometry_npatch": (_i32, [_vp]),
    "gf_geometry_destroy": (None, [_vp]),
    "gf_locate": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "gf_space_create": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, ctypes.POINTER(_vp)]),
    "gf_space_destroy": (None, [_vp]),
    "gf_space_ndofs": (_i64, [_vp]),
    "gf_space_noise_length": (_i64, [_vp]),
    "gf_space_dofmap": (_i32, [_vp, _vp]),
    "gf_space_apply": (_i32, [_vp, _dbl, _dbl, _i32, _vp, _vp, _i32, _i32]),
    "gf_space_transfer": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _i32]),
    "gf_space_cache_info": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                                   ctypes.POINTER(_i64)]),
    "gf_space_apply_noalloc": (_i32, [_vp, _dbl, _dbl, _i32, _vp, _vp, _i32]),
    "gf_white_noise": (_i32, [_vp, _i32, _vp, _vp, _i32]),
    "gf_sample": (_i32, [_vp, _dbl, _dbl, ctypes.POINTER(QuadRule), ctypes.POINTER(SolveOpts), _i32, _vp, _vp,
                         _i32, ctypes.POINTER(SolveStats)]),
    "gf_sample_batch": (_i32, [_vp, _i32, ctypes.POINTER(BatchItem), ctypes.POINTER(SolveOpts), _i32,
                               ctypes.POINTER(SolveStats)]),
    "gf_solve_shifted": (_i32, [_vp, _i32, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), _i32,
                                ctypes.POINTER(SolveStats)]),
    "gf_sqrt_mass_rule": (_i32, [_dbl, _dbl, _i32, _vp, _vp, ctypes.POINTER(_dbl)]),
    "gf_sqrt_mass": (_i32, [_vp, _i32, _vp, _vp, _i32, _dbl, _dbl, ctypes.POINTER(SolveOpts), _i32,
                            ctypes.POINTER(SolveStats)]),
    "gf_sample_tape": (_i32, [_vp, _dbl, _dbl, ctypes.POINTER(QuadRule), ctypes.POINTER(SolveOpts), _i32, _vp,
                              _vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(SolveStats)]),
    "gf_grad_kappa": (_i32, [_vp, _vp, _vp, _i32, ctypes.POINTER(SolveStats)]),
    "gf_tape_destroy": (None, [_vp]),
    "gf_eval": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _i32]),
    "gf_eval_adjoint": (_i32, [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _i32]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class GfieldError(RuntimeError):
    def __init__(self, status, msg, stats=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.stats = stats


def _check(status, stats=None):
    if status != GF_OK:
        raise GfieldError(status, _lib.gf_last_error().decode(), stats)


def abi_version():
    return _lib.gf_abi_version()


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _marshal_in(a, n):
    """(pointer, mem, keepalive) of a float64 input with n entries."""
    if _is_torch(a):
        import torch
        if a.dtype != torch.float64 or not a.is_cuda:
            raise TypeError("device arrays must be float64 CUDA tensors")
        a = a.contiguous()
        if a.numel() != n:
            raise ValueError(f"expected {n} entries, got {a.numel()}")
        return a.data_ptr(), GF_DEVICE, a
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"expected {n} entries, got {a.size}")
    return a.ctypes.data, GF_HOST, a


def _alloc_like(a, shape):
    if _is_torch(a):
        import torch
        return torch.empty(shape, dtype=torch.float64, device=a.device)
    return np.empty(shape, dtype=np.float64)


def _ptr(a):
    return a.data_ptr() if _is_torch(a) else a.ctypes.data


class Context:
    """One GPU and one HIP stream (torch's current stream on `device` when torch is given)."""

    def __init__(self, device=0, stream=None, use_torch_stream=True):
        h = _vp()
        s = stream
        if s is None and use_torch_stream:
            import torch
            s = torch.cuda.current_stream(device).cuda_stream
        _check(_lib.gf_context_create(device, s, ctypes.byref(h)))
        self.h = h
        self.device = device

    def probe_fma(self, precision=GF_PREC_FP64):
        """Achieved vector multiply-add rate of the device in TFLOP/s (FP64, or FP32 for
        GF_PREC_MIXED): measurement support for the roofline of the stencil kernels."""
        out = ctypes.c_double(0.0)
        _check(_lib.gf_probe_fma(self.h, precision, ctypes.byref(out)))
        return out.value

    def close(self):
        if self.h:
            _lib.gf_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# perturbation amplitude of the perturbed sphere of the batching workload
PERTURBED_AMP = 0.15


class Geometry:
    """The six-patch sphere family (gf_geometry_cubesphere; perturb_amp True stands for PERTURBED_AMP),
    or NURBS patches via Geometry.nurbs."""

    def __init__(self, ctx, perturb_amp=0.0, _handle=None):
        h = _handle
        if h is None:
            amp = PERTURBED_AMP if perturb_amp is True else float(perturb_amp)
            h = _vp()
            _check(_lib.gf_geometry_cubesphere(ctx.h if ctx is not None else None, amp, ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self.npatch = int(_lib.gf_geometry_npatch(h))

    @classmethod
    def nurbs(cls, ctx, deg_u, deg_v, ncoef, knots, ctrl):
        """NURBS patches in the layout of gf_geometry_nurbs (host arrays)."""
        nc = np.ascontiguousarray(ncoef, dtype=np.int32).reshape(-1, 2)
        kn = np.ascontiguousarray(knots, dtype=np.float64).reshape(-1)
        cp = np.ascontiguousarray(ctrl, dtype=np.float64).reshape(-1)
        h = _vp()
        _check(_lib.gf_geometry_nurbs(ctx.h if ctx is not None else None, len(nc), deg_u, deg_v, nc.ctypes.data,
                                      kn.ctypes.data, cp.ctypes.data, ctypes.byref(h)))
        return cls(ctx, _handle=h)

    def locate(self, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        n = len(xyz)
        patch = np.empty(n, dtype=np.int32)
        st = np.empty((n, 2), dtype=np.float64)
        _check(_lib.gf_locate(self.h, n, xyz.ctypes.data, patch.ctypes.data, st.ctypes.data))
        return patch, st

    def close(self):
        if self.h:
            _lib.gf_geometry_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Space:
    """S^0_{level,degree} on a geometry, with its multigrid hierarchy."""

    def __init__(self, ctx, geom, degree, level, nquad=0, mg_levels=0):
        h = _vp()
        _check(_lib.gf_space_create(ctx.h, geom.h, degree, level, nquad, mg_levels, ctypes.byref(h)))
        self.h = h
        self.ctx, self.geom = ctx, geom
        self.degree, self.level = degree, level
        self.ndofs = int(_lib.gf_space_ndofs(h))
        self.noise_length = int(_lib.gf_space_noise_length(h))

    def dofmap(self):
        n = 2 ** self.level + self.degree
        out = np.empty((self.geom.npatch, n, n), dtype=np.int32)
        _check(_lib.gf_space_dofmap(self.h, out.ctypes.data))
        return out

    def apply(self, sigma, s_scale, x, kind=GF_APPLY_STENCIL):
        """y = (sigma M + s_scale S) x for x of shape (nvec, N) or (N,)."""
        single = len(x.shape) == 1
        nvec = 1 if single else x.shape[0]
        px, mem, keep = _marshal_in(x, nvec * self.ndofs)
        y = _alloc_like(x, x.shape)
        _check(_lib.gf_space_apply(self.h, sigma, s_scale, nvec, px, _ptr(y), mem, kind))
        return y

    def transfer(self, level, direction, x, n_out):
        """Prolongation (GF_PROLONG: y = P x) or restriction (GF_RESTRICT: y = P^T x) between levels
        level-1 and level of the space's hierarchy; x of shape (nvec, n_in), n_out unknowns out."""
        single = len(x.shape) == 1
        nvec = 1 if single else x.shape[0]
        px, mem, keep = _marshal_in(x, nvec * x.shape[-1])
        y = _alloc_like(x, (n_out,) if single else (nvec, n_out))
        _check(_lib.gf_space_transfer(self.h, level, direction, nvec, px, _ptr(y), mem))
        return y

    def cache_info(self):
        """(plans, plan bytes, workspaces, workspace bytes) the space keeps cached for later calls."""
        n_p, b_p, n_w, b_w = _i32(), _i64(), _i32(), _i64()
        _check(_lib.gf_space_cache_info(self.h, ctypes.byref(n_p), ctypes.byref(b_p), ctypes.byref(n_w),
                                        ctypes.byref(b_w)))
        return n_p.value, b_p.value, n_w.value, b_w.value

    def apply_noalloc(self, sigma, s_scale, x, y, kind=GF_APPLY_STENCIL):
        """y = (sigma M + s_scale S) x into the preallocated device tensor y (nvec, N), queued on the
        context's stream without any device allocation."""
        if not (_is_torch(x) and _is_torch(y)):
            raise TypeError("x and y must be float64 CUDA tensors")
        nvec = 1 if len(x.shape) == 1 else x.shape[0]
        px, mem, keep = _marshal_in(x, nvec * self.ndofs)
        if y.dtype != x.dtype or not y.is_contiguous() or y.numel() != nvec * self.ndofs or y.device != x.device:
            raise ValueError("y must be a contiguous float64 tensor of the shape of x on its device")
        _check(_lib.gf_space_apply_noalloc(self.h, sigma, s_scale, nvec, px, y.data_ptr(), kind))
        return y

    def white_noise(self, z):
        """b = sum_e R_e^T L_e z_e for z of shape (nsamp, noise_length)."""
        nsamp = 1 if len(z.shape) == 1 else z.shape[0]
        pz, mem, keep = _marshal_in(z, nsamp * self.noise_length)
        b = _alloc_like(z, (nsamp, self.ndofs))
        _check(_lib.gf_white_noise(self.h, nsamp, pz, _ptr(b), mem))
        return b

    def sample(self, kappa, beta, b, h=0.4, k_minus=20, k_plus=20, precision=GF_PREC_FP64, rtol=1e-10,
               max_iter=500, cheb_degree=0, apply_kind=GF_APPLY_STENCIL, flags=0, split=GF_SPLIT_PLAIN,
               preconditioner=GF_PRECOND_VCYCLE):
        """Field samples u for loads b (nsamp, N); returns (u, stats dict)."""
        nsamp = 1 if len(b.shape) == 1 else b.shape[0]
        pb, mem, keep = _marshal_in(b, nsamp * self.ndofs)
        u = _alloc_like(b, (nsamp, self.ndofs))
        rule = QuadRule(h, k_minus, k_plus, split)
        opts = SolveOpts(precision, rtol, max_iter, cheb_degree, apply_kind, flags, preconditioner)
        st = SolveStats()
        status = _lib.gf_sample(self.h, kappa, beta, ctypes.byref(rule), ctypes.byref(opts), nsamp, pb, _ptr(u),
                                mem, ctypes.byref(st))
        _check(status, st.as_dict())
        return u, st.as_dict()

    def solve_shifted(self, sigma, b, precision=GF_PREC_FP64, rtol=1e-10, max_iter=500, cheb_degree=0,
                      apply_kind=GF_APPLY_STENCIL, flags=0, preconditioner=GF_PRECOND_VCYCLE):
        """x_i = (sigma_i M + S)^-1 b_i for b of shape (nsys, N); returns (x, stats dict)."""
        nsys = 1 if len(b.shape) == 1 else b.shape[0]
        sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (nsys,)))
        pb, mem, keep = _marshal_in(b, nsys * self.ndofs)
        x = _alloc_like(b, (nsys, self.ndofs))
        opts = SolveOpts(precision, rtol, max_iter, cheb_degree, apply_kind, flags, preconditioner)
        st = SolveStats()
        status = _lib.gf_solve_shifted(self.h, nsys, sig.ctypes.data, pb, _ptr(x), ctypes.byref(opts), mem,
                                       ctypes.byref(st))
        _check(status, st.as_dict())
        return x, st.as_dict()

    def sqrt_mass(self, y, khat=16, lo=0.0, hi=0.0, rtol=1e-12, max_iter=1000, flags=0):
        """f = sqrt(M) y for y of shape (nsamp, N) by the elliptic-function rule; returns (f, stats)."""
        nsamp = 1 if len(y.shape) == 1 else y.shape[0]
        py, mem, keep = _marshal_in(y, nsamp * self.ndofs)
        f = _alloc_like(y, (nsamp, self.ndofs))
        opts = SolveOpts(GF_PREC_FP64, rtol, max_iter, 0, GF_APPLY_STENCIL, flags)
        st = SolveStats()
        status = _lib.gf_sqrt_mass(self.h, nsamp, py, _ptr(f), khat, lo, hi, ctypes.byref(opts), mem,
                                   ctypes.byref(st))
        _check(status, st.as_dict())
        return f, st.as_dict()

    def sample_tape(self, kappa, beta, b, h=0.4, k_minus=20, k_plus=20, precision=GF_PREC_FP64, rtol=1e-10,
                    max_iter=500, cheb_degree=0, apply_kind=GF_APPLY_STENCIL, flags=0, split=GF_SPLIT_PLAIN,
                    preconditioner=GF_PRECOND_VCYCLE):
        """sample() that also keeps the forward solutions; returns (u, Tape, stats dict)."""
        nsamp = 1 if len(b.shape) == 1 else b.shape[0]
        pb, mem, keep = _marshal_in(b, nsamp * self.ndofs)
        u = _alloc_like(b, (nsamp, self.ndofs))
        rule = QuadRule(h, k_minus, k_plus, split)
        opts = SolveOpts(precision, rtol, max_iter, cheb_degree, apply_kind, flags, preconditioner)
        st = SolveStats()
        th = _vp()
        status = _lib.gf_sample_tape(self.h, kappa, beta, ctypes.byref(rule), ctypes.byref(opts), nsamp, pb,
                                     _ptr(u), mem, ctypes.byref(th), ctypes.byref(st))
        _check(status, st.as_dict())
        return u, Tape(th, self, nsamp), st.as_dict()

    def _points(self, patch, st, like):
        """patch (npts,) int32 and st (npts, 2) float64 in the memory kind of `like`."""
        if _is_torch(like):
            import torch
            patch = torch.as_tensor(patch, dtype=torch.int32, device=like.device).contiguous()
            st = torch.as_tensor(st, dtype=torch.float64, device=like.device).reshape(-1, 2).contiguous()
        else:
            patch = np.ascontiguousarray(patch, dtype=np.int32)
            st = np.ascontiguousarray(st, dtype=np.float64).reshape(-1, 2)
        if patch.shape[0] != st.shape[0]:
            raise ValueError("patch and st must describe the same points")
        return patch, st

    def eval(self, patch, st, u):
        """Point values Phi u: u (nvec, N) -> (nvec, npts)."""
        nvec = 1 if len(u.shape) == 1 else u.shape[0]
        pu, mem, keep = _marshal_in(u, nvec * self.ndofs)
        patch, st = self._points(patch, st, u)
        npts = patch.shape[0]
        vals = _alloc_like(u, (nvec, npts))
        _check(_lib.gf_eval(self.h, npts, _ptr(patch), _ptr(st), nvec, pu, _ptr(vals), mem))
        return vals

    def eval_adjoint(self, patch, st, r):
        """Phi^T r: r (nvec, npts) -> (nvec, N)."""
        patch, st = self._points(patch, st, r)
        npts = patch.shape[0]
        nvec = 1 if len(r.shape) == 1 else r.shape[0]
        pr, mem, keep = _marshal_in(r, nvec * npts)
        out = _alloc_like(r, (nvec, self.ndofs))
        _check(_lib.gf_eval_adjoint(self.h, npts, _ptr(patch), _ptr(st), nvec, pr, _ptr(out), mem))
        return out

    def close(self):
        if self.h:
            _lib.gf_space_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tape:
    """Forward state of one sample_tape call (keeps its space alive)."""

    def __init__(self, h, space, nsamp):
        self.h, self.space, self.nsamp = h, space, nsamp

    def grad_kappa(self, dl_du):
        """Per-sample dL_s/dkappa from dL/du (nsamp, N); returns (grad (nsamp,), stats dict)."""
        pg, mem, keep = _marshal_in(dl_du, self.nsamp * self.space.ndofs)
        out = _alloc_like(dl_du, (self.nsamp,))
        st = SolveStats()
        status = _lib.gf_grad_kappa(self.h, pg, _ptr(out), mem, ctypes.byref(st))
        _check(status, st.as_dict())
        return out, st.as_dict()

    def close(self):
        if self.h:
            _lib.gf_tape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sample_batch(ctx, requests, precision=GF_PREC_FP64, rtol=1e-10, max_iter=500, cheb_degree=0,
                 apply_kind=GF_APPLY_STENCIL, flags=0, preconditioner=GF_PRECOND_VCYCLE):
    """Several sampling requests solved together.

    requests: sequence of dicts with keys space, kappa, beta, b and optionally h, k_minus, k_plus,
    split (defaults 0.4, 20, 20, plain).  All loads must be of one kind (NumPy or CUDA tensors).
    Returns (list of u, stats dict)."""
    if not requests:
        raise ValueError("no requests")
    items = (BatchItem * len(requests))()
    keep, outs, mem0 = [], [], None
    for i, r in enumerate(requests):
        sp, b = r["space"], r["b"]
        nsamp = 1 if len(b.shape) == 1 else b.shape[0]
        pb, mem, kb = _marshal_in(b, nsamp * sp.ndofs)
        if mem0 is None:
            mem0 = mem
        elif mem != mem0:
            raise TypeError("all loads of a batch must be of one memory kind")
        u = _alloc_like(b, (nsamp, sp.ndofs))
        keep.append(kb)
        outs.append(u)
        items[i] = BatchItem(sp.h, r["kappa"], r["beta"],
                             QuadRule(r.get("h", 0.4), r.get("k_minus", 20), r.get("k_plus", 20),
                                      r.get("split", GF_SPLIT_PLAIN)), nsamp, pb,
                             _ptr(u))
    opts = SolveOpts(precision, rtol, max_iter, cheb_degree, apply_kind, flags, preconditioner)
    st = SolveStats()
    status = _lib.gf_sample_batch(ctx.h, len(requests), items, ctypes.byref(opts), mem0, ctypes.byref(st))
    _check(status, st.as_dict())
    return outs, st.as_dict()


def sqrt_mass_rule(lo, hi, khat):
    """(w2, a, c) of the square-root rule (host computation in the library)."""
    w2 = np.empty(khat)
    a = np.empty(khat)
    c = ctypes.c_double()
    _check(_lib.gf_sqrt_mass_rule(lo, hi, khat, w2.ctypes.data, a.ctypes.data, ctypes.byref(c)))
    return w2, a, c.value
