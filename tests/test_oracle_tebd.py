"""Pins of the oracle's TEBD propagation.

* untruncated TEBD equals a dense state vector driven by the same circuit;
* the Strang slice is second order: the error against exact piecewise-constant
  propagation drops 4x when dt halves;
* without renormalisation and truncation the norm is conserved and forward
  followed by the adjoint slices returns the input;
* the sweeps leave the canonical form they promise;
* with truncation the overlap error obeys the discarded-weight bound;
* transfer-matrix elements are invariant under bond gauges.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import grape, mps, statevector as sv, tebd


def _problem(**kw):
    base = dict(task="cnot", N=6, M=6, T=3.0, chi=64, K=2, R=2, seed=11)
    base.update(kw)
    return W.make_problem(**base)


@pytest.mark.parametrize("task,N", [("cnot", 6), ("x", 7), ("ghz", 6)])
def test_untruncated_tebd_equals_statevector(task, N):
    p = _problem(task=task, N=N, M=5, sigma=0.3)
    for k in range(p.K):
        for r in range(p.R):
            a = tebd.evolve(p, mps.product_state(p.inputs[r]), k)
            ref = sv.strang_states(p, k, sv.kron_vec(p.inputs[r]))[-1]
            assert np.abs(mps.to_dense(a) - ref).max() < 1e-12
            tgt = mps.to_dense(p.targets[r])
            assert abs(mps.overlap(p.targets[r], a) - np.vdot(tgt, ref)) < 1e-12


def test_strang_is_second_order():
    errs = []
    base = _problem(task="ghz", N=4, M=4, T=2.0, K=1, R=1, sigma=0.3, seed=3)
    for refine in (1, 2, 4):
        # same piecewise-constant controls, each slice cut into `refine` pieces
        p = dataclasses.replace(
            base, M=base.M * refine,
            ux=np.repeat(base.ux, refine, 0), uy=np.repeat(base.uy, refine, 0),
            uzz=np.repeat(base.uzz, refine, 0))
        psi0 = sv.kron_vec(base.inputs[0])
        approx = sv.strang_states(p, 0, psi0)[-1]
        exact = sv.exact_final(p, 0, psi0)
        errs.append(np.linalg.norm(approx - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs


def test_norm_and_unitarity_without_renormalisation():
    p = dataclasses.replace(_problem(N=8, M=6, sigma=0.5), renormalize=False)
    a0 = mps.product_state(p.inputs[1])
    states = tebd.evolve(p, a0, 1, keep_all=True)
    for a in states:
        assert abs(mps.norm(a) - 1.0) < 1e-12
    back = tebd.evolve(p, states[-1], 1, adjoint=True)
    assert abs(mps.overlap(a0, back) - 1.0) < 1e-12


@pytest.mark.parametrize("M", [3, 4])
def test_sweeps_leave_canonical_form(M):
    p = _problem(N=8, M=M, sigma=0.5)
    a = mps.product_state(p.inputs[0])
    # the last forward slice sweeps right to left, the one before it left to right
    assert not tebd.forward_ltr(p, M - 1) and tebd.forward_ltr(p, M - 2)
    a1 = tebd.forward_slice(p, a, M - 2, 0)      # left to right: centre at N-1
    assert all(mps.is_left_isometric(A) for A in a1[:-1])
    a2 = tebd.forward_slice(p, a1, M - 1, 0)     # right to left: centre at 0
    assert all(mps.is_right_isometric(A) for A in a2[1:])
    assert abs(np.linalg.norm(a2[0]) - 1.0) < 1e-13


def test_truncation_error_bound():
    p = _problem(task="ghz", N=10, M=12, T=6.0, chi=4, K=1, R=1, sigma=0.3, seed=5)
    exact = sv.strang_states(p, 0, sv.kron_vec(p.inputs[0]))[-1]
    stats = []
    a = tebd.evolve(p, mps.product_state(p.inputs[0]), 0, stats=stats)
    assert max(mps.bond_dims(a)) <= 4
    err = np.linalg.norm(mps.to_dense(a) - exact)
    w = np.array([s["discarded"] for s in stats])
    assert w.max() > 1e-8                        # truncation really active
    # one renormalised truncation moves the state by sqrt(w + (1-sqrt(1-w))^2)
    bound = np.sum(np.sqrt(w + (1.0 - np.sqrt(1.0 - w)) ** 2))
    assert err <= bound * (1 + 1e-9) + 1e-13


def test_truncation_keep_rule():
    S = np.array([1.0, 0.5, 1e-11, 0.999e-12, 1e-20])
    assert tebd.keep_count(S, 10, 1e-12) == 3
    assert tebd.keep_count(S, 2, 1e-12) == 2
    assert tebd.keep_count(np.array([0.0, 0.0]), 4, 1e-12) == 1


def test_transitions_are_gauge_invariant():
    rng = np.random.default_rng(7)
    p = _problem(N=6, M=4, sigma=0.4)
    a = tebd.evolve(p, mps.product_state(p.inputs[0]), 0)
    b = tebd.evolve(p, mps.right_canonicalize(p.targets[1]), 1, adjoint=True)

    def gauge(m):
        out = mps.copy(m)
        for j in range(len(out) - 1):
            D = out[j].shape[2]
            G = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)) + 3 * np.eye(D)
            out[j] = np.einsum("asb,bc->asc", out[j], G)
            out[j + 1] = np.einsum("cb,bsd->csd", np.linalg.inv(G), out[j + 1])
        return out

    E, F = grape.environments(b, a)
    rho = grape.transitions(b, a, E, F)
    ga, gb = gauge(a), gauge(b)
    E2, F2 = grape.environments(gb, ga)
    rho2 = grape.transitions(gb, ga, E2, F2)
    assert np.abs(rho - rho2).max() < 1e-12
    # and against dense single-site matrix elements
    av, bv = mps.to_dense(a), mps.to_dense(b)
    for j in range(p.N):
        for s in range(2):
            for t in range(2):
                G = np.zeros((2, 2), complex)
                G[s, t] = 1.0
                ref = np.vdot(bv, sv.apply_local(av, p.N, j, G))
                assert abs(rho[j, s, t] - ref) < 1e-12
