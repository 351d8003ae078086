"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Tolerance: 1e-10 relative at a fixed chi (fidelity, gradient, overlaps),
with an absolute floor of 1e-6 * |O| for per-trajectory overlaps.
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import grape as og, mps as omps, tebd as otebd  # noqa: E402

from gpu_helpers import device_problem, random_mps, rel  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03639_amd as P
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_overlap_uneven_dims(P):
    rng = np.random.default_rng(3)
    N = 9
    kets = [random_mps(rng, N, 6) for _ in range(6)]
    bras = [random_mps(rng, N, 5) for _ in range(3)]
    say("overlap: N=9, 6 kets x 3 bras")
    kb = P.MPSBatch.from_mps(kets, dcap=8)
    bb = P.MPSBatch.from_mps(bras, dcap=5)
    out = P.mps_overlap(bb, kb).cpu().numpy()
    ref = np.array([omps.overlap(bras[t % 3], kets[t]) for t in range(6)])
    assert rel(out, ref) < 1e-13


@pytest.mark.parametrize("task,N,M,chi,adjoint", [("x", 8, 6, 16, False), ("cnot", 8, 5, 16, False),
                                                   ("ghz", 10, 6, 4, False), ("cnot", 8, 5, 16, True)])
def test_evolve_matches_oracle(P, task, N, M, chi, adjoint):
    p = W.make_problem(task=task, N=N, M=M, T=M * 0.4, chi=chi, K=3, R=1, sigma=0.3, seed=17)
    say(f"evolve: task={task} N={N} M={M} chi={chi} adjoint={adjoint}")
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
        v, w = omps.to_dense(got[k]), omps.to_dense(ref)
        assert np.max(np.abs(v - w)) < 1e-12, (k, np.max(np.abs(v - w)))
    assert info["max_dim"] <= chi


def _grape_case(P, p, ckpt_stride=0, dcap=None):
    d = device_problem(p)
    res = P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                                d["targets"], dcap=dcap, ckpt_stride=ckpt_stride, want_traj_dO=True)
    torch.cuda.synchronize()
    return res


def cut_gaps(p, k, r):
    """Smallest relative gap sigma_k - sigma_{k+1} at cuts decided by chi, in
    the forward and in the backward propagation of trajectory (k, r)."""
    fw, bw = [], []
    otebd.evolve(p, omps.product_state(p.inputs[r]), k, stats=fw)
    otebd.evolve(p, omps.right_canonicalize(p.targets[r]), k, adjoint=True, stats=bw)
    return (min([s["gap"] for s in fw] + [np.inf]), min([s["gap"] for s in bw] + [np.inf]))


# Cases with active truncation are chosen so that no cut falls inside a
# near-degenerate pair of singular values (gap >= 1e-8 sigma_1, the reading of
# ties at the chi cut); the degenerate case is tested separately below.
@pytest.mark.parametrize("task,N,M,chi,sigma,seed", [
    ("x", 8, 12, 16, 0.02, 23), ("cnot", 8, 10, 16, 0.3, 23), ("ghz", 8, 9, 16, 0.3, 23),
    ("cnot", 10, 8, 4, 0.5, 25), ("ghz", 7, 7, 2, 0.5, 23), ("x", 10, 8, 3, 0.8, 28)])
def test_grape_matches_oracle(P, task, N, M, chi, sigma, seed):
    p = W.make_problem(task=task, N=N, M=M, T=M * 0.3, chi=chi, K=3, R=2, sigma=sigma, seed=seed)
    say(f"grape: task={task} N={N} M={M} chi={chi} seed={seed}")
    for k in range(p.K):
        for r in range(p.R):
            assert min(cut_gaps(p, k, r)) >= 1e-8
    res = _grape_case(P, p)
    ref = og.fidelity_grad(p, details=True)
    F = float(res["F"].cpu())
    assert abs(F - ref["F"]) <= 1e-10 * abs(ref["F"]) + 1e-15
    for name in ("g_ux", "g_uy", "g_uzz"):
        g = res[name].cpu().numpy()
        gr = ref[name]
        scale = max(np.max(np.abs(gr)), 1e-300)
        assert np.max(np.abs(g - gr)) <= 1e-10 * scale + 1e-15, (name, np.max(np.abs(g - gr)), scale)
    O = res["overlaps"].cpu().numpy()
    dO = res["traj_dO"].cpu().numpy()
    MN, MN1 = p.M * p.N, p.M * (p.N - 1)
    for k in range(p.K):
        for r in range(p.R):
            Or = ref["overlaps"][(k, r)]
            assert abs(O[k, r] - Or) <= 1e-10 * max(abs(Or), 1e-6)
            dux, duy, duzz = ref["dO"][(k, r)]
            t = k * p.R + r
            got = dO[t]
            refv = np.concatenate([dux.ravel(), duy.ravel(), duzz.ravel()])
            scale = max(np.max(np.abs(refv)), 1e-6)
            assert np.max(np.abs(got - refv)) <= 1e-10 * scale, (k, r)


def test_checkpoint_stride_is_bitwise_invariant(P):
    p = W.make_problem(task="cnot", N=8, M=11, T=3.0, chi=8, K=2, R=2, sigma=0.3, seed=5)
    say("checkpoint stride invariance")
    a = _grape_case(P, p, ckpt_stride=0)
    b = _grape_case(P, p, ckpt_stride=1)
    c = _grape_case(P, p, ckpt_stride=5)
    for name in ("F", "g_ux", "g_uy", "g_uzz"):
        assert torch.equal(a[name], b[name]), name
        assert torch.equal(a[name], c[name]), name


def test_capacity_bucket_growth(P):
    # dims reach 16 at N=8; a starting bucket of 8 overflows and is regrown
    p = W.make_problem(task="ghz", N=8, M=8, T=4.0, chi=16, K=2, R=1, sigma=0.5, seed=8)
    say("capacity growth")
    d = device_problem(p)
    P.tnrg._plan_cache.clear()
    res = P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                                d["targets"])
    ref = og.fidelity_grad(p)
    assert abs(float(res["F"].cpu()) - ref["F"]) <= 1e-10 * ref["F"]
    assert res["info"]["max_dim"] <= res["dcap"]


def test_degenerate_cut_compares_what_is_unique(P):
    """GHZ targets have exactly degenerate Schmidt values; with chi = 3 the
    backward cut splits a degenerate pair and several truncated states are
    equally correct.  The forward overlaps are unique where the forward cuts
    are not near-ties; the gradient must be finite and bounded."""
    p = W.make_problem(task="ghz", N=7, M=7, T=2.1, chi=3, K=3, R=2, sigma=0.5, seed=23)
    say("degenerate cut")
    res = _grape_case(P, p)
    ref = og.fidelity_grad(p)
    O = res["overlaps"].cpu().numpy()
    checked = 0
    for k in range(p.K):
        for r in range(p.R):
            fw, bw = cut_gaps(p, k, r)
            assert bw < 1e-12          # the backward cut is a genuine tie
            if fw >= 1e-8:
                Or = ref["overlaps"][(k, r)]
                assert abs(O[k, r] - Or) <= 1e-10 * max(abs(Or), 1e-6)
                checked += 1
    assert checked >= 1
    for name in ("g_ux", "g_uy", "g_uzz"):
        g = res[name].cpu().numpy()
        assert np.all(np.isfinite(g)) and np.max(np.abs(g)) < 10.0


# Capacities above 32 keep the bond-update working buffers in global scratch
# instead of LDS (a second compilation of the same kernels).
def test_global_scratch_variant_is_bitwise_the_lds_variant(P):
    p = W.make_problem(task="cnot", N=8, M=9, T=2.7, chi=64, K=2, R=2, sigma=0.3, seed=51)
    say("lds vs global-scratch variant: cnot N=8 (dims <= 16) at dcap 16, 64 and 128")
    lib = P.tnrg._lib
    try:
        for c in (16, 64, 128):
            assert lib.tnrg_plan_set_threads(c, 256) == 0
        a = _grape_case(P, p, dcap=16)
        b = _grape_case(P, p, dcap=64)
        c = _grape_case(P, p, dcap=128)
    finally:
        for cap in (16, 64, 128):
            lib.tnrg_plan_set_threads(cap, 0)
    assert (a["dcap"], b["dcap"], c["dcap"]) == (16, 64, 128)
    for name in ("F", "g_ux", "g_uy", "g_uzz", "overlaps", "traj_dO"):
        assert torch.equal(a[name], b[name]), name
        assert torch.equal(a[name], c[name]), name


@pytest.mark.parametrize("dcap", [64, 128])
def test_jacobi_in_lds_is_bitwise_the_global_one(P, dcap):
    """Capacities above 32: the Jacobi on an LDS copy of its matrix and on
    the global-scratch one give the same bits (ghz N = 12: bonds up to 64,
    ranks above and below the LDS limit at dcap 128)."""
    p = W.make_problem(task="ghz", N=12, M=8, T=5.0, chi=64, K=2, R=1, sigma=0.5, seed=31,
                       amp=2.0)
    say(f"jacobi in LDS vs global at dcap {dcap}")
    lib = P.tnrg._lib
    try:
        assert lib.tnrg_plan_set_jacobi_lds(0) == 0
        a = _grape_case(P, p, dcap=dcap)
        assert lib.tnrg_plan_set_jacobi_lds(1) == 0
        b = _grape_case(P, p, dcap=dcap)
    finally:
        lib.tnrg_plan_set_jacobi_lds(-1)
    assert lib.tnrg_plan_set_jacobi_lds(2) != 0
    for name in ("F", "g_ux", "g_uy", "g_uzz", "overlaps", "traj_dO"):
        assert torch.equal(a[name], b[name]), name


@pytest.mark.parametrize("N,M,T,chi,threads", [(12, 10, 6.0, 64, 0), (12, 10, 6.0, 64, 512)])
def test_large_bonds_match_oracle(P, N, M, T, chi, threads):
    """Bond dimensions above 32 (63 and 64, the full rank of the middle bond):
    the global-scratch variant against the oracle, with the default
    workgroup and with 512 threads."""
    p = W.make_problem(task="ghz", N=N, M=M, T=T, chi=chi, K=2, R=1, sigma=0.5, seed=31,
                       amp=2.0)
    say(f"large bonds: ghz N={N} M={M} chi={chi} threads={threads}")
    for k in range(p.K):
        assert min(cut_gaps(p, k, 0)) >= 1e-8
    lib = P.tnrg._lib
    try:
        assert lib.tnrg_plan_set_threads(64, threads) == 0
        res = _grape_case(P, p)
    finally:
        lib.tnrg_plan_set_threads(64, 0)
    assert lib.tnrg_plan_set_threads(16, 512) != 0
    assert res["dcap"] > 32 and res["info"]["max_dim"] > 32
    ref = og.fidelity_grad(p, details=True)
    F = float(res["F"].cpu())
    assert abs(F - ref["F"]) <= 1e-10 * abs(ref["F"])
    for name in ("g_ux", "g_uy", "g_uzz"):
        g = res[name].cpu().numpy()
        gr = ref[name]
        assert np.max(np.abs(g - gr)) <= 1e-10 * np.max(np.abs(gr)), name
    O = res["overlaps"].cpu().numpy()
    for (k, r), Or in ref["overlaps"].items():
        assert abs(O[k, r] - Or) <= 1e-10 * max(abs(Or), 1e-6)


# The paper's first-order split U_l = X_l Y_l Z_l (Sec. II, Eq. 4) with the
# insertions of App. A, against the oracle's first-order path.
@pytest.mark.parametrize("task,N,M,chi,sigma,seed", [
    ("x", 8, 12, 16, 0.02, 23), ("cnot", 8, 10, 16, 0.3, 23), ("ghz", 8, 9, 16, 0.3, 23),
    ("cnot", 10, 8, 4, 0.5, 25)])
def test_first_order_grape_matches_oracle(P, task, N, M, chi, sigma, seed):
    p = W.make_problem(task=task, N=N, M=M, T=M * 0.3, chi=chi, K=3, R=2, sigma=sigma, seed=seed,
                       order=1)
    say(f"first-order grape: task={task} N={N} M={M} chi={chi}")
    for k in range(p.K):
        for r in range(p.R):
            assert min(cut_gaps(p, k, r)) >= 1e-8
    res = _grape_case(P, p)
    ref = og.fidelity_grad(p, details=True)
    F = float(res["F"].cpu())
    assert abs(F - ref["F"]) <= 1e-10 * abs(ref["F"]) + 1e-15
    for name in ("g_ux", "g_uy", "g_uzz"):
        g = res[name].cpu().numpy()
        gr = ref[name]
        scale = max(np.max(np.abs(gr)), 1e-300)
        assert np.max(np.abs(g - gr)) <= 1e-10 * scale + 1e-15, (name, np.max(np.abs(g - gr)), scale)
    O = res["overlaps"].cpu().numpy()
    for (k, r), Or in ref["overlaps"].items():
        assert abs(O[k, r] - Or) <= 1e-10 * max(abs(Or), 1e-6)


@pytest.mark.parametrize("adjoint", [False, True])
def test_first_order_evolve_matches_oracle(P, adjoint):
    p = W.make_problem(task="cnot", N=8, M=5, T=2.0, chi=16, K=3, R=1, sigma=0.3, seed=17,
                       order=1)
    say(f"first-order evolve: adjoint={adjoint}")
    d = device_problem(p)
    states = [omps.product_state(p.inputs[0]) for _ in range(p.K)]
    if adjoint:
        states = [omps.right_canonicalize(p.targets[0]) for _ in range(p.K)]
    batch = P.MPSBatch.from_mps(states, dcap=16)
    P.mps_evolve(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], batch, adjoint=adjoint)
    got = batch.to_mps()
    for k in range(p.K):
        ref = otebd.evolve(p, states[k], k, adjoint=adjoint)
        assert np.max(np.abs(omps.to_dense(got[k]) - omps.to_dense(ref))) < 1e-12
