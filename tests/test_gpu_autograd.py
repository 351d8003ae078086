"""The forward/backward split of the persistent kernel and the
torch.autograd.Function over it.

  * grape_forward + grape_backward give the fused call's F and gradient bit
    for bit, and a backward without its forward is refused;
  * ensemble_fidelity(...).backward() puts the adjoint gradient on the
    control tensors, and matches the oracle;
  * at the full N = 50 CNOT workload (K = 128 noise samples x R = 8 inputs),
    the gradient from the autograd backward agrees with central differences
    (h = 1e-6) of the forward-only fidelity on 20 random control entries.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import grape as og  # noqa: E402

from gpu_helpers import device_problem  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from self_target import self_target  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03639_amd as P
    return P


def say(*a):
    print(*a, flush=True)


def test_split_equals_fused(P):
    p = W.make_problem(task="cnot", N=8, M=11, T=3.0, chi=8, K=3, R=2, sigma=0.3, seed=41)
    say("split vs fused: cnot N=8 M=11 chi=8")
    d = device_problem(p)
    args = (d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"], d["targets"])
    fused = P.grape_fidelity_grad(*args, dcap=8, want_traj_dO=True)
    call = P.tnrg.prepare(*args, dcap=8, want_traj_dO=True)
    F_fwd = call.F.clone()
    call.backward(d["ux"], d["uy"], d["uzz"], d["J"])
    call.check()
    assert torch.equal(F_fwd, fused["F"])
    assert torch.equal(call.overlaps.view(p.K, p.R), fused["overlaps"])
    for nm in ("g_ux", "g_uy", "g_uzz"):
        assert torch.equal(getattr(call, nm), fused[nm]), nm
    assert torch.equal(call.traj_dO, fused["traj_dO"])
    # a second backward from the same checkpoints gives the same result
    g1 = call.g_ux.clone()
    call.backward(d["ux"], d["uy"], d["uzz"], d["J"])
    call.check()
    assert torch.equal(call.g_ux, g1)


def test_backward_without_forward_is_refused(P):
    p = W.make_problem(task="x", N=6, M=5, T=2.0, chi=8, K=2, R=1, sigma=0.3, seed=42)
    say("stale backward")
    d = device_problem(p)
    call = P.GrapeCall(d["model"], p.K, p.R, d["inputs"], d["targets"], 8)
    call.ws.zero_()
    call.backward(d["ux"], d["uy"], d["uzz"], d["J"])
    info = call.check(raise_on_error=False)
    assert info["rc"] == P.tnrg.ESTALE
    assert np.all(info["flags"] == P.tnrg.FLAG_STALE)
    assert float(call.g_ux.abs().max()) == 0.0
    # a forward with other buffers does not validate this backward either
    call.forward(d["ux"], d["uy"], d["uzz"], d["J"])
    call.check()
    uy2 = d["uy"].clone()
    call.backward(d["ux"], uy2, d["uzz"], d["J"])
    assert call.check(raise_on_error=False)["rc"] == P.tnrg.ESTALE
    call.backward(d["ux"], d["uy"], d["uzz"], d["J"])
    assert call.check(raise_on_error=False)["rc"] == P.tnrg.OK


def test_autograd_matches_oracle(P):
    p = W.make_problem(task="cnot", N=8, M=9, T=2.7, chi=16, K=3, R=2, sigma=0.3, seed=43)
    say("autograd vs oracle: cnot N=8 M=9")
    d = device_problem(p)
    ux = d["ux"].clone().requires_grad_(True)
    uy = d["uy"].clone().requires_grad_(True)
    uzz = d["uzz"].clone().requires_grad_(True)
    F = P.ensemble_fidelity(d["model"], ux, uy, uzz, d["J"], d["inputs"], d["targets"])
    assert F.requires_grad and F.dim() == 0
    (3.0 * F).backward()
    ref = og.fidelity_grad(p)
    assert abs(float(F.detach()) - ref["F"]) <= 1e-10 * ref["F"]
    for t, nm in ((ux, "g_ux"), (uy, "g_uy"), (uzz, "g_uzz")):
        g = t.grad.cpu().numpy() / 3.0
        scale = np.max(np.abs(ref[nm]))
        assert np.max(np.abs(g - ref[nm])) <= 1e-10 * scale, nm
    with torch.no_grad():
        F2 = P.ensemble_fidelity(d["model"], ux, uy, uzz, d["J"], d["inputs"], d["targets"])
    assert float(F2) == float(F.detach())


def _fd_entries(p, rng, n):
    """n distinct random control entries (array, m, j); u^zz only on bonds
    that carry the control."""
    pool = [("ux", m, j) for m in range(p.M) for j in range(p.N)]
    pool += [("uy", m, j) for m in range(p.M) for j in range(p.N)]
    pool += [("uzz", m, b) for m in range(p.M) for b in range(p.N - 1) if p.zz_mask[b]]
    return [pool[i] for i in rng.choice(len(pool), size=n, replace=False)]


@pytest.mark.parametrize("self_tgt", [False, True])
def test_full_size_gradient_vs_central_differences(P, self_tgt):
    p = W.make_problem("cnot_n50")
    if self_tgt:
        p = self_target(p)
    say(f"central differences: cnot_n50 N={p.N} M={p.M} K={p.K} R={p.R} self_target={self_tgt}")
    d = device_problem(p)
    ux = d["ux"].clone().requires_grad_(True)
    uy = d["uy"].clone().requires_grad_(True)
    uzz = d["uzz"].clone().requires_grad_(True)
    F = P.ensemble_fidelity(d["model"], ux, uy, uzz, d["J"], d["inputs"], d["targets"])
    F.backward()
    grads = {"ux": ux.grad.cpu().numpy(), "uy": uy.grad.cpu().numpy(),
             "uzz": uzz.grad.cpu().numpy()}
    gmax = max(np.max(np.abs(g)) for g in grads.values())
    # forward-only evaluations reuse one prepared call and its workspace
    ctrl = {"ux": d["ux"].clone(), "uy": d["uy"].clone(), "uzz": d["uzz"].clone()}
    call = P.tnrg.prepare(d["model"], ctrl["ux"], ctrl["uy"], ctrl["uzz"], d["J"], d["inputs"],
                          d["targets"])
    F0 = float(call.F[0])
    assert F0 == float(F.detach())
    h = 1e-6
    rng = np.random.default_rng(2026)
    worst = 0.0
    for (nm, m, j) in _fd_entries(p, rng, 20):
        vals = []
        for sgn in (1.0, -1.0):
            ctrl[nm][m, j] += sgn * h
            call.forward(ctrl["ux"], ctrl["uy"], ctrl["uzz"], d["J"])
            call.check()
            vals.append(float(call.F[0]))
            ctrl[nm][m, j] -= sgn * h
        fd = (vals[0] - vals[1]) / (2 * h)
        g = float(grads[nm][m, j])
        err = abs(fd - g) / gmax
        worst = max(worst, err)
        say(f"  d/d{nm}[{m},{j}]: adjoint {g:+.9e} central {fd:+.9e} |diff|/|g|_inf {err:.1e}")
        # 1e-6 relative to the largest gradient entry, plus the rounding floor
        # of a central difference: F carries a relative rounding error of
        # about 1e-14 (the GPU-oracle agreement of O(1) overlaps), which
        # enters the difference quotient as 1e-14 F / h.  The floor matters
        # only when |grad| is small next to F (self-target, F ~ 0.4).
        assert abs(fd - g) <= 1e-6 * gmax + 1e-14 * F0 / h, (nm, m, j, g, fd)
    say(f"  F = {F0:.6e}, worst |diff| / |grad|_inf = {worst:.1e}")
