"""Robust GRAPE optimisation loop over the device kernels.

The paper optimises the ensemble fidelity with L-BFGS (Sec. II; the gradient
of App. A).  ``robust_grape`` does that with ``torch.optim.LBFGS`` on the
control tensors: every closure evaluation is one ``ensemble_fidelity``
forward (the forward kernel) and its backward (the adjoint kernel), so the
loop itself adds no computation of its own.  Bonds without a u^zz control
keep zero amplitude (their gradient is identically zero).
"""
from __future__ import annotations

from typing import Optional

import torch

from . import tnrg
from .autograd import ensemble_fidelity


def robust_grape(model: tnrg.Model, ux0, uy0, uzz0, J, inputs: tnrg.MPSBatch,
                 targets: tnrg.MPSBatch, iters: int = 50, dcap: Optional[int] = None,
                 ckpt_stride: int = 0, tol: float = 1e-12, history: Optional[list] = None):
    """Maximise F over (ux, uy, uzz) from the given start; returns the optimised
    controls (device float64 tensors) and the final fidelity.

    ``history`` (a list) receives the fidelity after every L-BFGS iteration.
    """
    dev = inputs.data.device
    ux = tnrg._f64(ux0, dev).clone().requires_grad_(True)
    uy = tnrg._f64(uy0, dev).clone().requires_grad_(True)
    uzz = tnrg._f64(uzz0, dev).clone().requires_grad_(True)
    J = tnrg._f64(J, dev)
    # one iteration per step() (for the history), with up to 25 line-search
    # evaluations (max_eval bounds the line search too)
    opt = torch.optim.LBFGS([ux, uy, uzz], lr=1.0, max_iter=1, max_eval=25, history_size=20,
                            tolerance_grad=tol, tolerance_change=tol,
                            line_search_fn="strong_wolfe")
    last = {}

    def closure():
        opt.zero_grad()
        F = ensemble_fidelity(model, ux, uy, uzz, J, inputs, targets, dcap, ckpt_stride)
        loss = 1.0 - F
        loss.backward()
        last["F"] = float(F.detach())
        return loss

    for _ in range(iters):
        opt.step(closure)
        if history is not None:
            history.append(last["F"])
    with torch.no_grad():
        F = float(ensemble_fidelity(model, ux, uy, uzz, J, inputs, targets, dcap, ckpt_stride))
    return dict(ux=ux.detach(), uy=uy.detach(), uzz=uzz.detach(), F=F)
