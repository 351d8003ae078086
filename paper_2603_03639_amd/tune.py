"""Launch-plan autotuner: workgroup size per capacity bucket, and the
checkpoint stride of the adjoint sweep under an HBM budget.

The persistent kernel runs one workgroup per trajectory.  With few
trajectories per SIMD the bond update is latency-bound, and 2 or 4 waves per
trajectory can hide latency better than one; which is fastest depends on the
bond dimensions the workload reaches.  ``autotune`` times each candidate on a
prefix of the caller's own problem (same N, capacity, ensemble size; long
enough for its bonds to reach half the capacity, within half the slices) and
stores the winner in the library's process-wide plan (tnrg_plan_set_threads).
Results do not depend on the choice beyond rounding.
"""
from __future__ import annotations

import time
from typing import Dict, Sequence

import torch

from . import tnrg

CANDIDATES = (64, 128, 256)
# capacities above 32 (global-scratch build) may also run 512 threads
BIG_CANDIDATES = (64, 128, 256, 512)
_tuned: Dict[tuple, int] = {}


def set_threads(dcap: int, threads: int) -> None:
    tnrg._check(tnrg._lib.tnrg_plan_set_threads(dcap, threads))


def threads(dcap: int) -> int:
    return int(tnrg._lib.tnrg_plan_threads(dcap))


def autotune(model: "tnrg.Model", ux, uy, uzz, J, inputs: "tnrg.MPSBatch",
             targets: "tnrg.MPSBatch", dcap: int, slices: int = 16,
             candidates: Sequence[int] = None, repeats: int = 1) -> dict:
    """Pick the fastest workgroup size for ``dcap`` on a prefix of the problem
    (the candidates default to CANDIDATES, BIG_CANDIDATES above capacity 32)."""
    if candidates is None:
        candidates = BIG_CANDIDATES if dcap > 32 else CANDIDATES
    K, R = int(J.shape[0]), inputs.n_traj
    key = (model.N, dcap, K * R, model.chi)
    if key in _tuned:
        set_threads(dcap, _tuned[key])
        return {"threads": _tuned[key], "cached": True}
    import dataclasses
    Ms = max(1, min(model.M, slices))
    # A prefix whose bonds stay far below the bucket times the small-bond
    # regime, where fewer threads win; lengthen it (doubling, up to half of
    # the slices) until its largest bond reaches half the capacity.
    while True:
        sub = dataclasses.replace(model, M=Ms)
        args = [a[:Ms].contiguous() for a in (ux, uy, uzz)] + [J]
        call = tnrg.GrapeCall(sub, K, R, inputs, targets, dcap, device=inputs.data.device)
        call.run(*args)
        torch.cuda.synchronize()
        reached = call.check()["max_dim"]
        del call
        if 2 * reached >= dcap or 2 * Ms > max(slices, model.M // 2):
            break
        Ms *= 2
    times = {}
    for nt in candidates:
        set_threads(dcap, nt)
        call = tnrg.GrapeCall(sub, K, R, inputs, targets, dcap, device=inputs.data.device)
        call.run(*args)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            call.run(*args)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        call.check()
        times[nt] = best
        del call
    win = min(times, key=times.get)
    set_threads(dcap, win)
    _tuned[key] = win
    return {"threads": win, "cached": False, "seconds": times, "slices": Ms,
            "prefix_max_dim": reached}


def ckpt_stride(model: "tnrg.Model", K: int, R: int, dcap: int, budget_bytes=None,
                frac: float = 0.6) -> dict:
    """Smallest checkpoint stride whose workspace fits the HBM budget.

    With stride s the forward pass keeps every s-th state and the adjoint
    sweep recomputes the states in between, (M - M/s) extra slices per
    trajectory; s = 1 keeps every forward state and recomputes nothing.  The
    default budget is ``frac`` of the device memory free now.  Returns the
    stride (0, the library's ceil(sqrt(M)), when even that does not fit) and
    the workspace bytes it needs.
    """
    if budget_bytes is None:
        free, _total = torch.cuda.mem_get_info()
        budget_bytes = int(frac * free)
    import math
    top = max(1, math.ceil(math.sqrt(model.M)))
    for s in range(1, top + 1):
        need = tnrg.grape_workspace_bytes(model, K, R, dcap, s)
        if need <= budget_bytes:
            return {"stride": s, "workspace_bytes": need, "budget_bytes": budget_bytes}
    return {"stride": 0, "workspace_bytes": tnrg.grape_workspace_bytes(model, K, R, dcap, 0),
            "budget_bytes": budget_bytes}
