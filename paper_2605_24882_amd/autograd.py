"""torch.autograd.Function wrappers of the sampler and of point evaluation.

`sample_field(kappa, b, space, beta, ...)` returns the field samples u (nsamp, N) as a function of a
0-dimensional float64 tensor kappa; its backward calls the library's adjoint (gf_grad_kappa), which
solves the adjoint shifted systems with the same batched solver, and returns dL/dkappa summed over
the samples.  `evaluate(u, space, patch, st)` returns the point values Phi u; its backward is
Phi^T (gf_eval_adjoint).  The load b is data (white noise): no gradient flows to it.

Arithmetic happens in the HIP library only; these classes move tensors and handles.
"""
import torch

from . import gfield as g


class SampleField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, b, space, beta, opts):
        if b.requires_grad:
            raise ValueError("the load b is not differentiable here; detach it")
        u, tape, st = space.sample_tape(float(kappa), beta, b.detach().contiguous(), **opts)
        ctx.tape = tape
        ctx.kappa_shape = kappa.shape
        ctx.stats = st
        return u

    @staticmethod
    def backward(ctx, grad_u):
        per_sample, _ = ctx.tape.grad_kappa(grad_u.contiguous())
        dk = per_sample.sum().reshape(ctx.kappa_shape)
        return dk, None, None, None, None


class EvaluateField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, space, patch, st):
        ctx.space, ctx.patch, ctx.st = space, patch, st
        return space.eval(patch, st, u.contiguous())

    @staticmethod
    def backward(ctx, grad_vals):
        return ctx.space.eval_adjoint(ctx.patch, ctx.st, grad_vals.contiguous()), None, None, None


def sample_field(kappa, b, space, beta, h=0.4, k_minus=20, k_plus=20, precision=g.GF_PREC_FP64, rtol=1e-10,
                 max_iter=500, cheb_degree=0, apply_kind=g.GF_APPLY_STENCIL, split=g.GF_SPLIT_PLAIN,
                 preconditioner=g.GF_PRECOND_VCYCLE):
    """Field samples u(kappa) for loads b (nsamp, N) on the GPU, differentiable in kappa (plain or
    improved split)."""
    opts = dict(h=h, k_minus=k_minus, k_plus=k_plus, precision=precision, rtol=rtol, max_iter=max_iter,
                cheb_degree=cheb_degree, apply_kind=apply_kind, split=split, preconditioner=preconditioner)
    return SampleField.apply(kappa, b, space, beta, opts)


def evaluate(u, space, patch, st):
    """Point values (nsamp, npts) of fields u (nsamp, N), differentiable in u."""
    return EvaluateField.apply(u, space, patch, st)
