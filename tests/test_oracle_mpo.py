"""Pins of the oracle's gate objective with MPO propagation (Sec. II,
Eqs. 5-6; oracle/mpo.py), each against the dense state-vector path
(oracle/statevector.py), which shares no operator code with it:

* the embedded identity, parallel-X and CNOT-pair MPOs are those operators;
* without truncation the evolved MPO is the dense propagator, whose columns
  are the evolved basis states, in both crosstalk models and both splits;
* F is |tr(U_T^dag U)/2^n|^2 of that dense propagator;
* the adjoint gradient agrees with central differences of the dense gate
  fidelity (no adjoint involved);
* the global pi pulse gives F = 1 and a zero gradient at N = 50;
* with J^x = J^y = 0 the Heisenberg path (mid-sweep u^zz insertions) gives
  the ZZ model's F and gradient (boundary insertions);
* under truncation the bond dimension stays at chi and the vector norm at 1.
"""
import copy
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import gates, mpo, mps, statevector as sv

X = np.array([[0, 1], [1, 0]], complex)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], complex)


def _p(**kw):
    base = dict(task="cnot", N=4, M=4, T=2.0, chi=64, K=2, R=1, sigma=0.3, seed=19,
                delta_j=0.3)
    base.update(kw)
    return W.make_problem(**base)


def _dense_U(p, k):
    """Columns U e_i from the state-vector circuit."""
    n = p.N
    cols = []
    for i in range(2 ** n):
        e = np.zeros(2 ** n, complex)
        e[i] = 1.0
        cols.append(sv.strang_states(p, k, e)[-1])
    return np.stack(cols, axis=1)


def _dense_target(task, n):
    if task == "x":
        U = np.ones((1, 1), complex)
        for _ in range(n):
            U = np.kron(U, X)
        return U
    U = np.ones((1, 1), complex)
    for _ in range(n // 2):
        U = np.kron(U, CNOT)
    if n % 2:
        U = np.kron(U, np.eye(2))
    return U


def _dense_F(p):
    UT = _dense_target(p.task, p.N)
    return np.mean([abs(np.trace(UT.conj().T @ _dense_U(p, k)) / 2 ** p.N) ** 2
                    for k in range(p.K)])


def test_embedded_operators():
    assert np.allclose(mpo.to_matrix(mpo.identity(3)), np.eye(8), atol=1e-15)
    for task, n in (("x", 3), ("cnot", 4), ("cnot", 5)):
        T = mpo.gate_target(task, n)
        assert np.allclose(mpo.to_matrix(T), _dense_target(task, n), atol=1e-15)
        assert abs(mps.norm(T) - 1.0) < 1e-15


@pytest.mark.parametrize("xt,order,M", [("zz", 2, 4), ("zz", 1, 3), ("heisenberg", 2, 3),
                                        ("heisenberg", 1, 4)])
def test_untruncated_mpo_is_the_dense_propagator(xt, order, M):
    p = _p(M=M, order=order, xt_model=xt)
    for k in range(p.K):
        U = mpo.to_matrix(mpo.evolve(p, k))
        assert np.abs(U - _dense_U(p, k)).max() < 1e-12
        assert np.abs(U.conj().T @ U - np.eye(2 ** p.N)).max() < 1e-12


@pytest.mark.parametrize("task,xt", [("cnot", "zz"), ("x", "heisenberg"), ("cnot", "heisenberg")])
def test_fidelity_is_the_trace_formula(task, xt):
    p = _p(task=task, xt_model=xt)
    assert abs(mpo.gate_fidelity_grad(p)["F"] - _dense_F(p)) < 1e-13


@pytest.mark.parametrize("task,xt,order", [("cnot", "zz", 2), ("cnot", "heisenberg", 2),
                                           ("cnot", "heisenberg", 1), ("x", "zz", 1)])
def test_adjoint_equals_dense_central_differences(task, xt, order):
    p = _p(task=task, xt_model=xt, order=order, M=3)
    res = mpo.gate_fidelity_grad(p)
    rng = np.random.default_rng(8)
    h = 1e-6
    picks = [("ux", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(3)]
    picks += [("uy", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(3)]
    picks += [("uzz", (l, int(b))) for l in range(p.M) for b in np.nonzero(p.zz_mask)[0]]
    for name, idx in picks:
        pp = copy.deepcopy(p)
        getattr(pp, name)[idx] += h
        pm = copy.deepcopy(p)
        getattr(pm, name)[idx] -= h
        fd = (_dense_F(pp) - _dense_F(pm)) / (2 * h)
        an = res["g_" + name][idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_pi_pulse_n50():
    p = W.make_problem(task="x", N=50, M=6, T=10.0, chi=4, K=2, R=1, seed=1, controls="zero",
                       crosstalk=0.0)
    p.ux[:] = math.pi / p.T
    res = mpo.gate_fidelity_grad(p)
    assert abs(res["F"] - 1.0) < 1e-13
    assert np.abs(res["g_ux"]).max() < 1e-12 and np.abs(res["g_uy"]).max() < 1e-12


def test_zz_limit_equals_zz_model():
    ph = _p(N=5, M=4, xt_model="heisenberg")
    ph.J[:, :, :2] = 0.0
    pz = dataclasses.replace(ph, xt_model="zz", J=ph.J[:, :, 2].copy())
    a, b = mpo.gate_fidelity_grad(ph), mpo.gate_fidelity_grad(pz)
    assert abs(a["F"] - b["F"]) < 1e-13
    for key in ("g_ux", "g_uy", "g_uzz"):
        assert np.abs(a[key] - b[key]).max() < 1e-12, key


def test_truncation_keeps_chi_and_unit_norm():
    p = _p(N=6, M=4, chi=3, xt_model="heisenberg")
    U = mpo.evolve(p, 0)
    assert max(A.shape[2] for A in U) <= 3
    assert abs(mps.norm(U) - 1.0) < 1e-12
    F = mpo.gate_fidelity_grad(p)["F"]
    assert 0.0 <= F <= 1.0
