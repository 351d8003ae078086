"""Robust GRAPE optimisation loop over the device kernels, and the paper's
sequential strategies around it (warm starts in n and in the error
strength, the two-stage ensemble).

The paper optimises the ensemble fidelity with L-BFGS (Sec. II; the gradient
of App. A).  ``robust_grape`` does that with ``torch.optim.LBFGS`` on the
control tensors: every closure evaluation is one ``ensemble_fidelity``
forward (the forward kernel) and its backward (the adjoint kernel), so the
loop itself adds no computation of its own.  Bonds without a u^zz control
keep zero amplitude (their gradient is identically zero).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
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


# ----------------------------------------------------------------------------
# Sequential optimisation (Sec. II): warm starts across system sizes and
# error strengths, and the two-stage ensemble.

def parasitic_count(model: tnrg.Model) -> int:
    """n_J, the number of unknown parasitic strengths: one per crosstalk bond
    in the ZZ model, three (J^x, J^y, J^z) with Heisenberg crosstalk."""
    xt = model.xt_mask if model.xt_mask is not None else np.zeros(model.N - 1)
    return int(np.count_nonzero(xt)) * (3 if model.xt_model == 1 else 1)


def extend_controls(ux, uy, uzz, n_new: int):
    """Initial guess for n_new qubits from a solution for fewer (Sec. II: the
    solution for n - 1 qubits seeds n).  The paper does not say how the
    added qubit is driven; here the old qubits keep their controls, each
    added qubit repeats the drive of the qubit two places before it and each
    added bond the u^zz of the bond two places before it, so alternating
    patterns (the CNOT pairs) continue.  Arrays are (M, N) and (M, N-1)."""
    ux = torch.as_tensor(ux)
    uy = torch.as_tensor(uy)
    uzz = torch.as_tensor(uzz)
    n = ux.shape[1]
    if n_new < n:
        raise ValueError(f"cannot shrink {n} qubits to {n_new}")

    def grow(a, width):
        cols = [a[:, j] for j in range(a.shape[1])]
        while len(cols) < width:
            cols.append(cols[-2] if len(cols) >= 2 else cols[-1])
        return torch.stack(cols, 1).contiguous()
    return grow(ux, n_new), grow(uy, n_new), grow(uzz, n_new - 1)


def robustness_steps(dj_target: float, step: float = 0.01):
    """Error strengths 0, step, 2 step, ... up to dj_target (Sec. II: the
    error-free solution seeds 1 %, which seeds 2 %, ...)."""
    k = int(round(dj_target / step))
    if k < 0 or abs(k * step - dj_target) > 1e-12:
        raise ValueError(f"{dj_target} is not a multiple of {step}")
    return [i * step for i in range(k + 1)]


def sequential(stages, make, ux0, uy0, uzz0, iters: int = 50, dcap: Optional[int] = None,
               ckpt_stride: int = 0, tol: float = 1e-12):
    """Optimise stage after stage (Sec. II).  ``make(stage)`` returns a dict
    with the stage's ``model``, ``J``, ``inputs`` and ``targets`` (device);
    the first stage starts from (ux0, uy0, uzz0), every later one from the
    previous stage's solution, extended with ``extend_controls`` when the
    stage has more qubits.  Returns one dict per stage: the stage, the
    fidelity at its starting controls (``F_start``), the optimised controls,
    ``F`` and the per-iteration ``history``."""
    ux, uy, uzz = ux0, uy0, uzz0
    out = []
    for st in stages:
        d = make(st)
        model = d["model"]
        dev = d["inputs"].data.device
        if tnrg._f64(ux, dev).shape[1] != model.N:
            ux, uy, uzz = extend_controls(ux, uy, uzz, model.N)
        ux, uy, uzz = (tnrg._f64(a, dev) for a in (ux, uy, uzz))
        F0, _ = tnrg.fidelity(model, ux, uy, uzz, d["J"], d["inputs"], d["targets"], dcap)
        hist = []
        res = robust_grape(model, ux, uy, uzz, d["J"], d["inputs"], d["targets"], iters, dcap,
                           ckpt_stride, tol, hist)
        out.append(dict(stage=st, F_start=float(F0), F=res["F"], ux=res["ux"], uy=res["uy"],
                        uzz=res["uzz"], history=hist))
        ux, uy, uzz = res["ux"], res["uy"], res["uzz"]
    return out


def two_stage(make_ensemble, ux0, uy0, uzz0, n_j: int, iters: int = 50,
              dcap: Optional[int] = None, ckpt_stride: int = 0, tol: float = 1e-12):
    """The paper's two-stage ensemble (Sec. II): optimise over K = 2 n_J
    noise samples, then estimate the mean fidelity on 5 K fresh ones.
    ``make_ensemble(K, stage)`` returns the problem dict (as for
    ``sequential``) with K noise samples, stage 0 for the optimisation and
    stage 1 for the estimate (a different draw).  Returns the optimised
    controls, the training fidelity ``F_train`` and the estimate
    ``F_eval`` with its ensemble size."""
    k_train = 2 * n_j
    d = make_ensemble(k_train, 0)
    res = robust_grape(d["model"], ux0, uy0, uzz0, d["J"], d["inputs"], d["targets"], iters,
                       dcap, ckpt_stride, tol)
    e = make_ensemble(5 * k_train, 1)
    F, _ = tnrg.fidelity(e["model"], res["ux"], res["uy"], res["uzz"], e["J"], e["inputs"],
                         e["targets"], dcap)
    return dict(ux=res["ux"], uy=res["uy"], uzz=res["uzz"], F_train=res["F"], F_eval=float(F),
                K_train=k_train, K_eval=5 * k_train)
