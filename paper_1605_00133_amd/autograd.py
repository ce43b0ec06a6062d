"""The measurement operator f = C A p0 as a differentiable torch function.

The gradient of any loss of f with respect to p0 is the exact adjoint of the
discrete operator applied to the loss gradient, A^T C^T g (eq. BP, Sec. 4.4),
which pat_adjoint computes. So the backward tapes nothing: it needs the memory
of one application, whatever the number of time steps, and no checkpointing.
Gradients with respect to the operator's own parameters (sound speed, grid)
are not provided. Both directions run in the library's kernels; this module
only allocates the outputs and loops over a batch.
"""

import torch

from . import pat as P


class _Measure(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0, plan):
        ctx.plan = plan
        x = p0.detach().contiguous()
        f = torch.empty((x.shape[0],) + tuple(plan.data_shape), dtype=torch.float32, device=x.device)
        for b in range(x.shape[0]):
            P.pat_forward(plan, x[b], f[b])
        return f

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        g = g.contiguous()
        grad = torch.empty((g.shape[0],) + tuple(plan.vol_shape), dtype=torch.float32, device=g.device)
        for b in range(g.shape[0]):
            P.pat_adjoint(plan, g[b], grad[b])
        return grad, None


def measure(plan, p0):
    """f = C A p0 for one volume [nz, ny, nx] or a batch [B, nz, ny, nx]
    (float32, on the plan's device); differentiable in p0, backward A^T C^T.
    Returns [nt, mc] or [B, nt, mc]."""
    if p0.dim() not in (3, 4):
        raise ValueError(f"p0 must be [nz, ny, nx] or [B, nz, ny, nx], got shape {tuple(p0.shape)}")
    single = p0.dim() == 3
    f = _Measure.apply(p0.unsqueeze(0) if single else p0, plan)
    return f[0] if single else f
