"""Pins of the oracle's Heisenberg-type crosstalk (Sec. III, Eq. 9:
J^x XX + J^y YY + J^z ZZ on every bond, J uniform in [-dJ, dJ], Sec. II).

* the bond gate is the 4x4 exponential, checked against its closed form on
  the {00, 11} and {01, 10} blocks, and is the ZZ phase when J^x = J^y = 0;
* the dense circuit is the product of the exponentials of the pieces, bonds
  in sweep order, built here from scratch;
* the alternating sweep order keeps the split at second order against exact
  propagation (a fixed bond order would be first order);
* untruncated TEBD equals the dense circuit and its adjoint undoes it;
* the adjoint gradient, with the mid-sweep u^zz insertions, agrees with
  central differences of the dense circuit's fidelity (no adjoint involved);
* with J^x = J^y = 0 the Heisenberg code path gives the ZZ model's F and
  gradient, which come from the boundary insertions (a different route).
"""
import copy
import dataclasses

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import workloads as W
from oracle import gates, grape, mps, statevector as sv, tebd

X = np.array([[0, 1], [1, 0]], complex)
Y = np.array([[0, -1j], [1j, 0]])
Zm = np.diag([1.0, -1.0]).astype(complex)


def _p(**kw):
    base = dict(task="cnot", N=5, M=4, T=2.0, chi=64, K=2, R=2, seed=71,
                xt_model="heisenberg", delta_j=0.3)
    base.update(kw)
    return W.make_problem(**base)


def test_noise_draw():
    p = W.make_problem(task="cnot", N=10, M=4, K=500, R=1, seed=3, xt_model="heisenberg",
                       delta_j=0.05)
    assert p.J.shape == (500, 9, 3)
    assert p.xt_mask.all() and np.abs(p.J).max() <= 0.05
    # uniform on [-dJ, dJ]: mean 0, variance dJ^2 / 3
    assert abs(p.J.mean()) < 3e-3 and abs(p.J.var() / (0.05 ** 2 / 3) - 1) < 0.05


@pytest.mark.parametrize("jx,jy,cz,dt", [(0.3, -0.2, 0.7, 0.4), (1.1, 0.9, -0.5, 0.05),
                                         (0.0, 0.0, 0.4, 0.3), (-0.6, 0.6, 0.0, 1.0)])
def test_bond_gate_closed_form(jx, jy, cz, dt):
    G = gates.bond_gate(jx, jy, cz, dt).reshape(4, 4)
    # XX and YY swap |00> <-> |11> with signs +, - and |01> <-> |10> with +, +,
    # and ZZ is +1 on the first pair, -1 on the second
    ref = np.zeros((4, 4), complex)
    for (i, j), a, z in (((0, 3), jx - jy, cz), ((1, 2), jx + jy, -cz)):
        ph = np.exp(-1j * dt * z)
        ref[i, i] = ref[j, j] = ph * np.cos(dt * a)
        ref[i, j] = ref[j, i] = -1j * ph * np.sin(dt * a)
    assert np.abs(G - ref).max() < 1e-14
    if jx == 0 and jy == 0:
        assert np.abs(np.diag(G).reshape(2, 2) - gates.zz_phase(dt * cz)).max() < 1e-14


def _site(op, j, N):
    return scipy.sparse.kron(scipy.sparse.identity(2 ** j),
                             scipy.sparse.kron(op, scipy.sparse.identity(2 ** (N - j - 1))))


def _bond(op4, b, N):
    return scipy.sparse.kron(scipy.sparse.identity(2 ** b),
                             scipy.sparse.kron(op4, scipy.sparse.identity(2 ** (N - b - 2))))


def _h_bond(p, k, l, b):
    J = p.J[k][b]
    c = p.zz_mask[b] * p.uzz[l, b] + J[2]
    return _bond(J[0] * np.kron(X, X) + J[1] * np.kron(Y, Y) + c * np.kron(Zm, Zm), b, p.N).tocsc()


def _h_drive(p, l):
    return sum(_site(0.5 * (p.ux[l, j] * X + p.uy[l, j] * Y), j, p.N) for j in range(p.N)).tocsc()


@pytest.mark.parametrize("M", [3, 4])
def test_dense_circuit_is_the_ordered_product_of_exponentials(M):
    p = _p(N=4, M=M)
    psi0 = sv.kron_vec(p.inputs[0])
    got = sv.strang_states(p, 1, psi0)[-1]
    psi = psi0.copy()
    for l in range(p.M):
        Hd = _h_drive(p, l)
        psi = scipy.sparse.linalg.expm_multiply(-0.5j * p.dt * Hd, psi)
        # the last slice visits the bonds right to left, the one before left
        # to right, and so on backwards in time
        ltr = (p.M - 1 - l) % 2 == 1
        for b in (range(p.N - 1) if ltr else range(p.N - 2, -1, -1)):
            psi = scipy.sparse.linalg.expm_multiply(-1j * p.dt * _h_bond(p, 1, l, b), psi)
        psi = scipy.sparse.linalg.expm_multiply(-0.5j * p.dt * Hd, psi)
    assert np.abs(got - psi).max() < 1e-12


def test_alternating_bond_order_is_second_order():
    base = _p(task="ghz", N=4, M=2, T=1.0, K=1, R=1, seed=3)
    psi0 = sv.kron_vec(base.inputs[0])
    H = _h_drive(base, 0) + sum(_h_bond(base, 0, 0, b) for b in range(base.N - 1))
    exact = scipy.sparse.linalg.expm_multiply(-1j * base.T * H, psi0)
    errs = []
    for M in (8, 16, 32):
        p = dataclasses.replace(base, M=M, ux=np.repeat(base.ux[:1], M, 0),
                                uy=np.repeat(base.uy[:1], M, 0),
                                uzz=np.repeat(base.uzz[:1], M, 0))
        errs.append(np.linalg.norm(sv.strang_states(p, 0, psi0)[-1] - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs


@pytest.mark.parametrize("task,N,M,order", [("cnot", 6, 5, 2), ("x", 7, 4, 2), ("ghz", 6, 5, 1),
                                            ("cnot", 5, 4, 1)])
def test_untruncated_tebd_equals_statevector(task, N, M, order):
    p = _p(task=task, N=N, M=M, order=order)
    for k in range(p.K):
        a = tebd.evolve(p, mps.product_state(p.inputs[0]), k)
        ref = sv.strang_states(p, k, sv.kron_vec(p.inputs[0]))[-1]
        assert np.abs(mps.to_dense(a) - ref).max() < 1e-12
        b = tebd.evolve(p, a, k, adjoint=True)
        assert np.abs(mps.to_dense(b) - sv.kron_vec(p.inputs[0])).max() < 1e-12


def _dense_F(q):
    tot = 0.0
    for k in range(q.K):
        for r in range(q.R):
            a = sv.strang_states(q, k, sv.kron_vec(q.inputs[r]))[-1]
            tot += abs(np.vdot(mps.to_dense(q.targets[r]), a)) ** 2
    return tot / (q.K * q.R)


@pytest.mark.parametrize("task,M,order", [("cnot", 4, 2), ("ghz", 3, 2), ("cnot", 3, 1)])
def test_adjoint_equals_dense_central_differences(task, M, order):
    p = _p(task=task, N=5, M=M, K=2, R=1, order=order)
    res = grape.fidelity_grad(p)
    rng = np.random.default_rng(5)
    h = 1e-6
    zz_bonds = np.nonzero(p.zz_mask)[0]
    picks = [("ux", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(3)]
    picks += [("uy", (int(rng.integers(p.M)), int(rng.integers(p.N)))) for _ in range(3)]
    picks += [("uzz", (l, int(b))) for l in range(p.M) for b in zz_bonds]
    for name, idx in picks:
        pp = copy.deepcopy(p)
        getattr(pp, name)[idx] += h
        pm = copy.deepcopy(p)
        getattr(pm, name)[idx] -= h
        fd = (_dense_F(pp) - _dense_F(pm)) / (2 * h)
        an = res["g_" + name][idx]
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


@pytest.mark.parametrize("task,M,order", [("cnot", 4, 2), ("ghz", 5, 2), ("cnot", 5, 1)])
def test_zz_limit_equals_zz_model(task, M, order):
    ph = _p(task=task, N=6, M=M, K=2, R=2, order=order)
    ph.J[:, :, :2] = 0.0
    pz = dataclasses.replace(ph, xt_model="zz", J=ph.J[:, :, 2].copy(),
                             xt_mask=np.ones(ph.N - 1, np.uint8))
    rh = grape.fidelity_grad(ph)
    rz = grape.fidelity_grad(pz)
    assert abs(rh["F"] - rz["F"]) < 1e-13
    for key in ("g_ux", "g_uy", "g_uzz"):
        assert np.abs(rh[key] - rz[key]).max() < 1e-12, key
