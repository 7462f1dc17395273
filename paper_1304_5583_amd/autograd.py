"""torch.autograd.Function around dfc_lrr_solve / dfc_lrr_backward.

``dfc_lrr(Mt, lam, perm, offsets, opts)`` returns ``Zt`` (an (n, n) tensor
holding the column-major Z, as ``binding.dfc_lrr_solve``) and records the
unrolled forward (``opts.fixed_iters`` iterations, checkpoints every
``opts.checkpoint_every``) on the context, so that ``Zt.backward(...)`` or
``torch.autograd.grad`` returns gradients with respect to ``Mt`` and to
``lam`` (a 0-d float64 tensor).  The reverse sweep replays the checkpointed
segments; it consumes the record, so one forward supports one backward, and any
other solve on the same context in between invalidates it (LRR_ENOTAPE).
"""
from __future__ import annotations

import torch

from . import binding as B


class DFCLRRFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, Mt, lam, perm, offsets, opts, ctx):
        opts = B.lrr_opts_default() if opts is None else opts
        if opts.fixed_iters <= 0:
            raise ValueError("the differentiable solve is the unrolled map: set opts.fixed_iters > 0")
        opts.save_for_backward = 1
        Zt, _, info = B.dfc_lrr_solve(Mt, float(lam), perm, offsets, opts=opts, ctx=ctx, want_S=False)
        fctx.m = Mt.shape[1]
        fctx.ctx = ctx or B.get_context(Mt.device.index or 0)
        fctx.info = info
        return Zt

    @staticmethod
    def backward(fctx, dZt):
        dlam, dMt = B.dfc_lrr_backward(dZt.contiguous(), ctx=fctx.ctx, want_dM=True, m=fctx.m)
        return dMt, torch.tensor(dlam, dtype=torch.float64, device=dZt.device), None, None, None, None


def dfc_lrr(Mt, lam, perm, offsets, opts=None, ctx=None):
    """Differentiable Algorithm 1 (unrolled, fixed iteration count)."""
    if not torch.is_tensor(lam):
        lam = torch.tensor(float(lam), dtype=torch.float64, device=Mt.device)
    return DFCLRRFunction.apply(Mt, lam, perm, offsets, opts, ctx)
