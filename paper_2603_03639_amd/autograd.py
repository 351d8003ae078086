"""torch.autograd.Function over the persistent kernels.

``ensemble_fidelity`` returns the ensemble fidelity F (Sec. II, Eq. 7) as a
0-dim float64 tensor whose graph reaches the control tensors ux, uy, uzz.
The forward pass runs only the forward propagation (grape_forward), keeping
the sqrt(M) checkpoints in a workspace owned by the graph node; the backward
pass runs the adjoint-sweep kernel (grape_backward, App. A) on them and
scales the gradient by the incoming grad_output.  A graph that never calls
backward pays for the forward propagation alone.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import tnrg


class EnsembleFidelity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ux, uy, uzz, J, model, inputs, targets, dcap, ckpt_stride):
        dev = inputs.data.device
        args = [tnrg._f64(a.detach(), dev) for a in (ux, uy, uzz, J)]
        call = tnrg.prepare(model, *args, inputs, targets, dcap, ckpt_stride)
        ctx.call = call
        ctx.args = args
        # saved so that autograd rejects a backward after an in-place change
        # of the controls (the checkpoints belong to the old values)
        ctx.save_for_backward(ux, uy, uzz, J)
        return call.F[0].clone()

    @staticmethod
    def backward(ctx, gF):
        ctx.saved_tensors  # noqa: B018  (raises if a control changed in place)
        call, args = ctx.call, ctx.args
        call.backward(*args)
        call.check()
        ctx.call = ctx.args = None  # release the workspace with the graph
        # bonds without a u^zz control get a zero gradient from the kernel
        return (gF * call.g_ux, gF * call.g_uy, gF * call.g_uzz, None, None, None, None, None,
                None)


def ensemble_fidelity(model: tnrg.Model, ux: torch.Tensor, uy: torch.Tensor,
                      uzz: torch.Tensor, J: torch.Tensor, inputs: tnrg.MPSBatch,
                      targets: tnrg.MPSBatch, dcap: Optional[int] = None,
                      ckpt_stride: int = 0) -> torch.Tensor:
    """F(ux, uy, uzz) for the ensemble J[K][N-1] x R inputs, differentiable in
    the controls (float64 tensors [M][N], [M][N], [M][N-1] on the device)."""
    return EnsembleFidelity.apply(ux, uy, uzz, J, model, inputs, targets, dcap, ckpt_stride)
