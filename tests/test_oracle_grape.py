"""Pins of the oracle's fidelity and adjoint gradient.

* adjoint gradient == gradient of the dense Strang circuit (N <= 7);
* adjoint gradient == central finite differences of the oracle itself (h=1e-6);
* the global pi pulse realises the parallel X gate with F = 1 and grad F = 0
  at N = 50 when the crosstalk is off (Sec. III);
* pure-ZZ evolution of |+>^N has F = prod_b cos^2(J_b T) and
  dF/du^zz_{l,b} = -2 dt tan(J_b T) F at N = 50;
* with the ZZ layer off the chain factorises into N qubits, whose overlaps and
  derivatives are plain 2x2 products (N = 50).
"""
import copy
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import gates, grape, mps, statevector as sv


@pytest.mark.parametrize("task", ["cnot", "ghz", "x"])
def test_adjoint_equals_dense_gradient(task):
    p = W.make_problem(task=task, N=6, M=5, T=2.5, chi=64, K=2, R=2, sigma=0.3, seed=21)
    for k, r in [(0, 0), (1, 1)]:
        O, dux, duy, duzz = grape.trajectory(p, k, r)
        O2, dux2, duy2, duzz2 = sv.adjoint_gradient(
            p, k, sv.kron_vec(p.inputs[r]), mps.to_dense(p.targets[r]))
        assert abs(O - O2) < 1e-12
        for a, b in [(dux, dux2), (duy, duy2), (duzz, duzz2)]:
            assert np.abs(a - b).max() < 1e-11


def test_adjoint_equals_central_differences():
    p = W.make_problem(task="cnot", N=6, M=4, T=2.0, chi=64, K=2, R=1, sigma=0.3, seed=4)
    res = grape.fidelity_grad(p)
    rng = np.random.default_rng(0)
    h = 1e-6
    picks = [("ux", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(4)]
    picks += [("uy", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(4)]
    picks += [("uzz", (int(rng.integers(p.M)), 2 * int(rng.integers(p.N // 2)))) for _ in range(4)]
    for name, idx in picks:
        pp = copy.deepcopy(p)
        getattr(pp, name)[idx] += h
        pm = copy.deepcopy(p)
        getattr(pm, name)[idx] -= h
        fd = (grape.fidelity_grad(pp)["F"] - grape.fidelity_grad(pm)["F"]) / (2 * h)
        an = res["g_" + name][idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_pi_pulse_parallel_x_gate_n50():
    p = W.make_problem(task="x", N=50, M=10, T=10.0, chi=32, K=2, R=2, seed=1,
                       controls="zero", crosstalk=0.0)
    p.ux[:] = math.pi / p.T
    res = grape.fidelity_grad(p)
    assert abs(res["F"] - 1.0) < 1e-13
    assert np.abs(res["g_ux"]).max() < 1e-12
    assert np.abs(res["g_uy"]).max() < 1e-12
    for O in res["overlaps"].values():
        assert abs(O - (-1j) ** 50) < 1e-12


def _zz_problem(N, M, T, seed):
    p = W.make_problem(task="ghz", N=N, M=M, T=T, chi=8, K=2, R=1, sigma=0.1,
                       seed=seed, controls="zero")
    plus = np.full((1, N, 2), 2 ** -0.5, complex)
    return dataclasses.replace(p, inputs=plus,
                               targets=[mps.product_state(plus[0])])


def test_pure_zz_closed_form_n50():
    p = _zz_problem(N=50, M=4, T=2.0, seed=9)
    res = grape.fidelity_grad(p, details=True)
    for k in range(p.K):
        J = p.J[k]
        O = res["overlaps"][(k, 0)]
        assert abs(O - np.prod(np.cos(J * p.T))) < 1e-13
        dux, duy, duzz = res["dO"][(k, 0)]
        # dO/du^zz_{l,b} = -dt tan(J_b T) O for every slice l
        ref = -p.dt * np.tan(J * p.T) * O
        assert np.abs(duzz - ref[None, :]).max() < 1e-13
    F = np.mean([np.prod(np.cos(p.J[k] * p.T) ** 2) for k in range(p.K)])
    assert abs(res["F"] - F) < 1e-13
    gz = np.mean([-2 * p.dt * np.tan(p.J[k] * p.T) * np.prod(np.cos(p.J[k] * p.T) ** 2)
                  for k in range(p.K)], axis=0)
    assert np.abs(res["g_uzz"] - gz[None, :]).max() < 1e-13


def test_independent_qubits_closed_form_n50():
    p = W.make_problem(task="x", N=50, M=6, T=3.0, chi=16, K=1, R=2, seed=8,
                       crosstalk=0.0)
    res = grape.fidelity_grad(p, details=True)
    dt = p.dt
    for r in range(p.R):
        # per qubit: o_j = <t_j| prod_l R_{l,j}^2 |in_j>
        o = np.zeros(p.N, complex)
        do_x = np.zeros((p.M, p.N), complex)
        do_y = np.zeros((p.M, p.N), complex)
        for j in range(p.N):
            Rs = [gates.half_rotation(p.ux[l, j], p.uy[l, j], dt) for l in range(p.M)]
            dRs = [gates.half_rotation_derivs(p.ux[l, j], p.uy[l, j], dt) for l in range(p.M)]
            tj = p.targets[r][j].reshape(2)
            ij = p.inputs[r, j]

            def chain(l_star=None, which=None):
                v = ij.copy()
                for l in range(p.M):
                    if l == l_star:
                        d = dRs[l][which]
                        v = (d @ Rs[l] + Rs[l] @ d) @ v
                    else:
                        v = Rs[l] @ (Rs[l] @ v)
                return np.vdot(tj, v)
            o[j] = chain()
            for l in range(p.M):
                do_x[l, j] = chain(l, 0)
                do_y[l, j] = chain(l, 1)
        O = np.prod(o)
        assert abs(res["overlaps"][(0, r)] - O) < 1e-13
        dux, duy, _ = res["dO"][(0, r)]
        rest = np.array([np.prod(np.delete(o, j)) for j in range(p.N)])
        assert np.abs(dux - do_x * rest[None, :]).max() < 1e-13
        assert np.abs(duy - do_y * rest[None, :]).max() < 1e-13
