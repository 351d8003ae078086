"""Pins of the oracle's first-order split (the X Y Z product of Sec. II,
Eq. 4, with the gradient insertions of App. A).

* the X and Y factors are the matrix exponentials of the drive terms, and
  their derivatives agree with central differences;
* the dense first-order circuit equals the product of the matrix
  exponentials of the three Hamiltonian pieces, built here from scratch;
* the split is first order: the error against exact propagation halves when
  dt halves;
* untruncated TEBD with the first-order split equals the dense circuit;
* the adjoint gradient agrees with central differences of the dense
  circuit's fidelity (an independent computation: no adjoint involved);
* the global pi pulse gives F = 1 and grad F = 0 at N = 50.
"""
import copy
import dataclasses
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import workloads as W
from oracle import gates, grape, mps, statevector as sv, tebd


def _p(**kw):
    base = dict(task="cnot", N=5, M=4, T=2.0, chi=64, K=2, R=2, sigma=0.3, seed=71, order=1)
    base.update(kw)
    return W.make_problem(**base)


@pytest.mark.parametrize("ux,uy,dt", [(0.7, -0.3, 0.2), (-1.3, 0.9, 0.05), (0.0, 0.4, 0.5)])
def test_first_order_factors_are_exponentials(ux, uy, dt):
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]])
    ref = scipy.linalg.expm(-0.5j * dt * ux * X) @ scipy.linalg.expm(-0.5j * dt * uy * Y)
    assert np.abs(gates.first_order_rotation(ux, uy, dt) - ref).max() < 1e-14
    h = 1e-6
    dx, dy = gates.first_order_rotation_derivs(ux, uy, dt)
    fdx = (gates.first_order_rotation(ux + h, uy, dt) - gates.first_order_rotation(ux - h, uy, dt)) / (2 * h)
    fdy = (gates.first_order_rotation(ux, uy + h, dt) - gates.first_order_rotation(ux, uy - h, dt)) / (2 * h)
    assert np.abs(dx - fdx).max() < 1e-9 and np.abs(dy - fdy).max() < 1e-9


def _pieces(p, k, l):
    """Sparse H_x, H_y, H_zz of slice l (qubit 0 is the most significant
    factor of the Kronecker products, as in the oracle's dense vectors)."""
    N = p.N
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]])
    Zm = np.diag([1.0, -1.0]).astype(complex)

    def site(op, j):
        return scipy.sparse.kron(scipy.sparse.identity(2 ** j),
                                 scipy.sparse.kron(op, scipy.sparse.identity(2 ** (N - j - 1))))
    Hx = sum(site(0.5 * p.ux[l, j] * X, j) for j in range(N))
    Hy = sum(site(0.5 * p.uy[l, j] * Y, j) for j in range(N))
    c = p.zz_mask * p.uzz[l] + p.xt_mask * p.J[k]
    Hz = sum(c[b] * site(Zm, b) @ site(Zm, b + 1) for b in range(N - 1))
    return Hx.tocsc(), Hy.tocsc(), Hz.tocsc()


def test_dense_first_order_circuit_is_the_product_of_exponentials():
    p = _p(N=4, M=3)
    psi0 = sv.kron_vec(p.inputs[0])
    got = sv.strang_states(p, 1, psi0)[-1]
    psi = psi0.copy()
    for l in range(p.M):
        Hx, Hy, Hz = _pieces(p, 1, l)
        psi = scipy.sparse.linalg.expm_multiply(-1j * p.dt * Hz, psi)
        psi = scipy.sparse.linalg.expm_multiply(-1j * p.dt * Hy, psi)
        psi = scipy.sparse.linalg.expm_multiply(-1j * p.dt * Hx, psi)
    assert np.abs(got - psi).max() < 1e-12


def test_first_order_split_is_first_order():
    base = _p(task="ghz", N=4, M=4, T=2.0, K=1, R=1, seed=3)
    errs = []
    for refine in (4, 8, 16):
        p = dataclasses.replace(
            base, M=base.M * refine,
            ux=np.repeat(base.ux, refine, 0), uy=np.repeat(base.uy, refine, 0),
            uzz=np.repeat(base.uzz, refine, 0))
        psi0 = sv.kron_vec(base.inputs[0])
        errs.append(np.linalg.norm(sv.strang_states(p, 0, psi0)[-1] - sv.exact_final(p, 0, psi0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.9 < r2 < 2.1, errs


@pytest.mark.parametrize("task,N", [("cnot", 6), ("x", 7), ("ghz", 6)])
def test_untruncated_first_order_tebd_equals_statevector(task, N):
    p = _p(task=task, N=N, M=5)
    for k in range(p.K):
        a = tebd.evolve(p, mps.product_state(p.inputs[0]), k)
        ref = sv.strang_states(p, k, sv.kron_vec(p.inputs[0]))[-1]
        assert np.abs(mps.to_dense(a) - ref).max() < 1e-12
        b = tebd.evolve(p, a, k, adjoint=True)
        assert np.abs(mps.to_dense(b) - sv.kron_vec(p.inputs[0])).max() < 1e-12


def test_first_order_adjoint_equals_dense_central_differences():
    p = _p(N=5, M=4, K=2, R=1)
    res = grape.fidelity_grad(p)

    def dense_F(q):
        tot = 0.0
        for k in range(q.K):
            for r in range(q.R):
                a = sv.strang_states(q, k, sv.kron_vec(q.inputs[r]))[-1]
                tot += abs(np.vdot(mps.to_dense(q.targets[r]), a)) ** 2
        return tot / (q.K * q.R)
    rng = np.random.default_rng(5)
    h = 1e-6
    picks = [("ux", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(4)]
    picks += [("uy", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(4)]
    picks += [("uzz", (int(rng.integers(p.M)), 2 * int(rng.integers(p.N // 2)))) for _ in range(3)]
    for name, idx in picks:
        pp = copy.deepcopy(p)
        getattr(pp, name)[idx] += h
        pm = copy.deepcopy(p)
        getattr(pm, name)[idx] -= h
        fd = (dense_F(pp) - dense_F(pm)) / (2 * h)
        an = res["g_" + name][idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_first_order_pi_pulse_n50():
    p = W.make_problem(task="x", N=50, M=10, T=10.0, chi=32, K=2, R=2, seed=1,
                       controls="zero", crosstalk=0.0, order=1)
    p.ux[:] = math.pi / p.T
    res = grape.fidelity_grad(p)
    assert abs(res["F"] - 1.0) < 1e-13
    assert np.abs(res["g_ux"]).max() < 1e-12 and np.abs(res["g_uy"]).max() < 1e-12
