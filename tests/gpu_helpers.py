"""Shared helpers for the GPU tests: marshal a seeded Problem to the device."""
import numpy as np
import torch

import paper_2603_03639_amd as P
from oracle import mps as omps


def device_problem(p, dev="cuda"):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=dev)
    inputs = P.MPSBatch.from_product(p.inputs, device=dev)
    tcap = max(max(A.shape[0] for A in T) for T in p.targets)
    targets = P.MPSBatch.from_mps(p.targets, dcap=max(1, tcap), device=dev)
    return dict(model=P.Model.from_problem(p), ux=f(p.ux), uy=f(p.uy), uzz=f(p.uzz), J=f(p.J),
                inputs=inputs, targets=targets)


def random_mps(rng, N, dmax):
    dims = [1] + [int(rng.integers(1, min(dmax, 2 ** min(j, N - j)) + 1)) for j in range(1, N)] + [1]
    return [(rng.standard_normal((dims[j], 2, dims[j + 1]))
             + 1j * rng.standard_normal((dims[j], 2, dims[j + 1]))) / np.sqrt(2 * dims[j + 1])
            for j in range(N)]


def rel(a, b, floor=0.0):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), floor, 1e-300))
