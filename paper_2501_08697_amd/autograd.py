"""torch.autograd.Function over the library's H psi and its hand-written adjoint.

forward  y = H(V, D) psi                       (abacus_pw_apply_h)
backward grad_psi, grad_V, grad_D from dY       (abacus_pw_apply_h_backward)

The adjoint recomputes the real-space grids from psi and dY; nothing but the
inputs is saved for backward. Gradients follow PyTorch's convention for
complex tensors (dL/dRe + i dL/dIm for a real loss L).
"""
from __future__ import annotations

import torch

from . import binding


class PwApplyH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, vloc, dmat, dp, precision):
        psi, vloc, dmat = psi.contiguous(), vloc.contiguous(), dmat.contiguous()
        y = binding.apply_h(dp, psi, precision, vloc=vloc, dmat=dmat)
        ctx.save_for_backward(psi, vloc, dmat)
        ctx.dp = dp
        ctx.precision = precision
        return y

    @staticmethod
    def backward(ctx, gy):
        psi, vloc, dmat = ctx.saved_tensors
        need = ctx.needs_input_grad
        want = tuple(n for n, w in zip(("psi", "v", "d"), need[:3]) if w)
        gp, gv, gd = binding.apply_h_backward(ctx.dp, psi, gy.contiguous(), ctx.precision, want=want,
                                              vloc=vloc, dmat=dmat)
        return gp, gv, gd, None, None


def apply_h(dp: binding.DeviceProblem, psi, vloc=None, dmat=None, precision: int = binding.FP64):
    """Differentiable H psi with respect to psi, V_loc(r) and the D blocks."""
    vloc = dp.vloc if vloc is None else vloc
    dmat = dp.dmat if dmat is None else dmat
    return PwApplyH.apply(psi, vloc, dmat, dp, precision)
