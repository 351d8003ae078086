"""Self-target variant of a workload (test infrastructure; uses the oracle).

With random controls at N = 50 the overlaps <T_r|a_M> of the gate targets are
1e-7 or smaller, so relative comparisons there say little about the states.
The self-target variant keeps the workload's controls, crosstalk samples and
inputs, and replaces each target T_r by the noise-free (J = 0) truncated
evolution of input r under the same controls, right-canonicalised with unit
norm.  The overlaps are then O(1) and shrink only through the crosstalk.
"""
import dataclasses

import numpy as np

from oracle import mps as omps, tebd as otebd


def self_target(p):
    quiet = dataclasses.replace(p, J=np.zeros((1,) + p.J.shape[1:]))
    targets = []
    for r in range(p.R):
        a = otebd.evolve(quiet, omps.product_state(p.inputs[r]), 0)
        targets.append(omps.right_canonicalize(a))
    return dataclasses.replace(p, targets=targets, name=p.name + "_self")


def golden_problem(name):
    """The problem a full-size sample name stands for: a workload name, then
    optionally "_heisenberg" (the paper's XX + YY + ZZ crosstalk instead of
    the workload's ZZ one) and "_self" (the self-target variant)."""
    import workloads as W
    self_t = name.endswith("_self")
    n = name[:-len("_self")] if self_t else name
    heis = n.endswith("_heisenberg")
    base = n[:-len("_heisenberg")] if heis else n
    p = W.make_problem(base, xt_model="heisenberg" if heis else "zz")
    return (self_target(p) if self_t else p), base
