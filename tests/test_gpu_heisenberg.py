"""GPU parity with the paper's Heisenberg-type crosstalk (Sec. III, Eq. 9):
the HIP library against the CPU oracle on the same seeded inputs.

The two-site layer is the product of 4x4 bond exponentials in sweep order,
and with u^zz controls the adjoint takes the u^zz derivative inside its
sweeps (a separate kernel instance).  Tolerance as in the other parity
tests: 1e-10 relative at a fixed chi.
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import grape as og, mps as omps, tebd as otebd  # noqa: E402

from gpu_helpers import device_problem  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03639_amd as P
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(task, N, M, chi, seed, order=2, K=3, R=2, dj=0.3):
    return W.make_problem(task=task, N=N, M=M, T=M * 0.3, chi=chi, K=K, R=R, seed=seed,
                          order=order, xt_model="heisenberg", delta_j=dj)


def _grape(P, p, ckpt_stride=0, dcap=None):
    d = device_problem(p)
    res = P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                                d["targets"], dcap=dcap, ckpt_stride=ckpt_stride, want_traj_dO=True)
    torch.cuda.synchronize()
    return res


def _min_gap(p):
    g = np.inf
    for k in range(p.K):
        for r in range(p.R):
            for adj, st0 in ((False, omps.product_state(p.inputs[r])),
                             (True, omps.right_canonicalize(p.targets[r]))):
                stats = []
                otebd.evolve(p, st0, k, adjoint=adj, stats=stats)
                g = min([g] + [s["gap"] for s in stats])
    return g


def _compare(res, ref, p):
    F = float(res["F"].cpu())
    assert abs(F - ref["F"]) <= 1e-10 * abs(ref["F"]) + 1e-15
    for name in ("g_ux", "g_uy", "g_uzz"):
        g = res[name].cpu().numpy()
        gr = ref[name]
        scale = max(np.max(np.abs(gr)), 1e-300)
        assert np.max(np.abs(g - gr)) <= 1e-10 * scale + 1e-15, (name, np.max(np.abs(g - gr)), scale)
    O = res["overlaps"].cpu().numpy()
    dO = res["traj_dO"].cpu().numpy()
    for k in range(p.K):
        for r in range(p.R):
            Or = ref["overlaps"][(k, r)]
            assert abs(O[k, r] - Or) <= 1e-10 * max(abs(Or), 1e-6)
            dux, duy, duzz = ref["dO"][(k, r)]
            refv = np.concatenate([dux.ravel(), duy.ravel(), duzz.ravel()])
            scale = max(np.max(np.abs(refv)), 1e-6)
            assert np.max(np.abs(dO[k * p.R + r] - refv)) <= 1e-10 * scale, (k, r)


@pytest.mark.parametrize("task,N,M,chi,adjoint,order", [
    ("cnot", 8, 5, 16, False, 2), ("cnot", 8, 6, 16, True, 2), ("x", 9, 4, 16, False, 1),
    ("ghz", 8, 5, 4, True, 2)])
def test_evolve_matches_oracle(P, task, N, M, chi, adjoint, order):
    p = _problem(task, N, M, chi, 17, order=order, R=1)
    say(f"heisenberg evolve: task={task} N={N} M={M} chi={chi} adjoint={adjoint} order={order}")
    d = device_problem(p)
    states = [omps.product_state(p.inputs[0]) for _ in range(p.K)]
    if adjoint:
        states = [omps.right_canonicalize(p.targets[0]) for _ in range(p.K)]
    batch = P.MPSBatch.from_mps(states, dcap=chi)
    info = P.mps_evolve(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], batch, adjoint=adjoint)
    got = batch.to_mps()
    for k in range(p.K):
        ref = otebd.evolve(p, states[k], k, adjoint=adjoint)
        assert omps.bond_dims(got[k]) == omps.bond_dims(ref)
        assert np.max(np.abs(omps.to_dense(got[k]) - omps.to_dense(ref))) < 1e-12, k
    assert info["max_dim"] <= chi


# cnot and ghz carry u^zz controls (mid-sweep insertions), x does not; odd
# and even M (the sweep direction rule), both splits, truncation at chi = 4,
# and checkpoint strides 1, 3 (not dividing M) and the default.
@pytest.mark.parametrize("task,N,M,chi,seed,order,stride", [
    ("cnot", 8, 10, 16, 23, 2, 0), ("cnot", 8, 9, 16, 24, 2, 1), ("ghz", 8, 9, 16, 23, 2, 3),
    ("x", 8, 8, 16, 23, 2, 0), ("cnot", 10, 8, 4, 25, 2, 0), ("cnot", 8, 7, 16, 26, 1, 2),
    ("ghz", 9, 8, 16, 27, 1, 1)])
def test_grape_matches_oracle(P, task, N, M, chi, seed, order, stride):
    p = _problem(task, N, M, chi, seed, order=order)
    say(f"heisenberg grape: task={task} N={N} M={M} chi={chi} seed={seed} order={order} "
        f"stride={stride}")
    assert _min_gap(p) >= 1e-8
    res = _grape(P, p, ckpt_stride=stride)
    _compare(res, og.fidelity_grad(p, details=True), p)


def test_checkpoint_stride_is_bitwise_invariant(P):
    p = _problem("cnot", 8, 11, 8, 5, K=2)
    say("heisenberg checkpoint stride invariance")
    a = _grape(P, p, ckpt_stride=0)
    b = _grape(P, p, ckpt_stride=1)
    c = _grape(P, p, ckpt_stride=5)
    for name in ("F", "g_ux", "g_uy", "g_uzz", "traj_dO"):
        assert torch.equal(a[name], b[name]), name
        assert torch.equal(a[name], c[name]), name


def test_global_scratch_variant_is_bitwise_the_lds_variant(P):
    p = _problem("cnot", 8, 9, 64, 51, K=2)
    say("heisenberg lds vs global-scratch variant at dcap 16 and 64")
    lib = P.tnrg._lib
    try:
        for c in (16, 64):
            assert lib.tnrg_plan_set_threads(c, 256) == 0
        a = _grape(P, p, dcap=16)
        b = _grape(P, p, dcap=64)
    finally:
        for cap in (16, 64):
            lib.tnrg_plan_set_threads(cap, 0)
    assert (a["dcap"], b["dcap"]) == (16, 64)
    for name in ("F", "g_ux", "g_uy", "g_uzz", "overlaps", "traj_dO"):
        assert torch.equal(a[name], b[name]), name


def test_zz_limit_equals_zz_model(P):
    """J^x = J^y = 0: the Heisenberg kernels (bond gates, mid-sweep u^zz
    insertions) against the ZZ-model kernels (phases, boundary insertions)."""
    ph = _problem("cnot", 10, 8, 16, 33)
    ph.J[:, :, :2] = 0.0
    pz = dataclasses.replace(ph, xt_model="zz", J=ph.J[:, :, 2].copy())
    say("heisenberg zz limit vs zz model")
    a = _grape(P, ph)
    b = _grape(P, pz)
    assert abs(float(a["F"]) - float(b["F"])) <= 1e-13
    for name in ("g_ux", "g_uy", "g_uzz"):
        x, y = a[name].cpu().numpy(), b[name].cpu().numpy()
        assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(y)), name


def test_autograd_split_equals_fused_call(P):
    """grape_forward + grape_backward (the autograd path) give the fused
    call's gradient bit for bit with the mid-sweep insertions."""
    p = _problem("cnot", 8, 6, 16, 41, K=2)
    say("heisenberg autograd vs fused")
    d = device_problem(p)
    fused = _grape(P, p)
    ux, uy, uzz = (d[k].clone().requires_grad_(True) for k in ("ux", "uy", "uzz"))
    F = P.ensemble_fidelity(d["model"], ux, uy, uzz, d["J"], d["inputs"], d["targets"])
    F.backward()
    torch.cuda.synchronize()
    assert torch.equal(F.detach().reshape(1), fused["F"].reshape(1))
    assert torch.equal(ux.grad, fused["g_ux"])
    assert torch.equal(uy.grad, fused["g_uy"])
    assert torch.equal(uzz.grad, fused["g_uzz"])


def test_wrong_crosstalk_shape_is_rejected(P):
    p = _problem("cnot", 6, 4, 8, 3, K=2)
    d = device_problem(p)
    with pytest.raises(ValueError):
        P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"][:, :, 2].contiguous(),
                              d["inputs"], d["targets"])
