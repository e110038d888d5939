"""The CV map as a differentiable PyTorch operation.

PySAGES differentiates its CVs with JAX (Sec. 2 and Sec. 2.2).  Here the
forward pass is the library's CV kernels and the backward pass is its
hand-written vector-Jacobian product (``sx_cv_vjp``: pos_bar = J^T xi_bar,
recomputed from the positions in gather form), so any bias written as a
torch function of xi -- a harmonic restraint k/2 (xi - xi0)^2 (Sec. 2.1.1),
a surrogate network -- yields atom forces through autograd.
"""
import torch


class CVFunction(torch.autograd.Function):
    """xi = CVFunction.apply(pos, sampler): (W, D) float64 CV values of the
    positions ``pos`` (device tensor in the sampler's layout, float32 or
    float64) for a bound :class:`~paper_2301_04835_amd.api.Sampler`."""

    @staticmethod
    def forward(ctx, pos, sampler, layout="aos3"):
        xi, _ = sampler.eval_cv(pos.detach(), jac=False, layout=layout)
        ctx.save_for_backward(pos.detach())
        ctx.sampler = sampler
        ctx.layout = layout
        return xi

    @staticmethod
    def backward(ctx, xi_bar):
        (pos,) = ctx.saved_tensors
        pos_bar = torch.zeros(pos.shape, dtype=torch.float32, device=pos.device)
        ctx.sampler.cv_vjp(pos, xi_bar.detach().to(torch.float64).contiguous(), pos_bar, layout=ctx.layout)
        return pos_bar.to(pos.dtype), None, None


def cv(pos, sampler, layout="aos3"):
    """Differentiable CV values (see :class:`CVFunction`)."""
    return CVFunction.apply(pos, sampler, layout)
