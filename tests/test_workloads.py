"""Seeded inputs: determinism, masks, canonical targets, task definitions."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import mps, statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_seeded_and_deterministic():
    a = W.make_problem("cnot_n50")
    b = W.make_problem("cnot_n50")
    for f in ("ux", "uy", "uzz", "J", "inputs"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert (a.N, a.M, a.K, a.R, a.chi) == (50, 200, 128, 8, 64)
    assert abs(a.dt - 0.05) < 1e-15


def test_cnot_masks_and_crosstalk():
    p = W.make_problem("cnot_n50")
    assert np.all(p.zz_mask[0::2] == 1) and np.all(p.zz_mask[1::2] == 0)
    assert np.all(p.xt_mask == 1 - p.zz_mask)
    assert np.all(p.J[:, 0::2] == 0) and np.all(p.uzz[:, 1::2] == 0)
    s = p.J[:, 1::2].std()
    assert 0.017 < s < 0.023          # Normal(0, 0.02), sigma = std dev


@pytest.mark.parametrize("name", ["xgate_n8", "cnot_n50", "ghz_n30"])
def test_targets_right_canonical_unit_norm(name):
    p = W.make_problem(name, K=1)
    for T in p.targets:
        assert all(mps.is_right_isometric(A) for A in T[1:])
        assert abs(np.linalg.norm(T[0]) - 1.0) < 1e-14


def test_cnot_target_is_pairwise_cnot():
    p = W.make_problem(task="cnot", N=6, M=2, K=1, R=2, seed=3)
    cnot = np.eye(4)[[0, 1, 3, 2]]
    for r in range(p.R):
        ref = np.ones(1, complex)
        for q in range(p.N // 2):
            ref = np.kron(ref, cnot @ np.kron(p.inputs[r, 2 * q], p.inputs[r, 2 * q + 1]))
        assert np.abs(mps.to_dense(p.targets[r]) - ref).max() < 1e-14


def test_x_target_is_flipped_input():
    p = W.make_problem(task="x", N=5, M=2, K=1, R=1, seed=3)
    X = np.array([[0, 1], [1, 0]])
    ref = sv.kron_vec([X @ v for v in p.inputs[0]])
    assert np.abs(mps.to_dense(p.targets[0]) - ref).max() < 1e-15


def test_ghz_mps_matches_paper_fixture():
    g = json.load(open(os.path.join(GOLDEN, "ghz_mps_sec4.json")))
    T = W.ghz_mps(g["n"])
    assert np.allclose(T[0].reshape(-1), np.array(g["first_site"]).reshape(-1))
    assert np.allclose(T[1][:, 0, :], g["middle_site_s0"])
    assert np.allclose(T[1][:, 1, :], g["middle_site_s1"])
    assert np.allclose(T[-1].reshape(2, 2), np.array(g["last_site"]).reshape(2, 2))
    v = mps.to_dense(T)
    ref = np.zeros(2 ** g["n"])
    for idx, amp in g["nonzero_amplitudes"].items():
        ref[int(idx)] = amp
    assert np.abs(v - ref).max() < 1e-15
    assert abs(mps.norm(W.ghz_mps(30)) - 1.0) < 1e-14


# ----------------------------------------------------------------------------
# Heisenberg ground-state target of the serving mix (state preparation,
# Sec. IV): Lanczos in the S^z = 0 sector, compressed to an MPS.
def _dense_heisenberg(N):
    X = np.array([[0, 1], [1, 0]], complex)
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1.0, -1.0]).astype(complex)
    H = np.zeros((2 ** N, 2 ** N), complex)
    for j in range(N - 1):
        for P in (X, Y, Z):
            ops = [np.eye(2)] * N
            ops[j] = P
            ops[j + 1] = P
            # bit j of the index is qubit j: the kron order runs from qubit
            # N-1 (most significant) down to qubit 0
            M = np.array([[1.0]])
            for q in range(N - 1, -1, -1):
                M = np.kron(M, ops[q])
            H += M
    return H.real


@pytest.mark.parametrize("N", [6, 8, 10])
def test_heisenberg_ground_state_is_the_dense_one(N):
    psi, E = W.heisenberg_ground_state(N)
    w, v = np.linalg.eigh(_dense_heisenberg(N))
    assert abs(E - w[0]) < 1e-10 * abs(w[0])
    assert w[1] - w[0] > 1e-3                     # non-degenerate (singlet)
    assert abs(abs(np.dot(v[:, 0], psi)) - 1.0) < 1e-10
    H = _dense_heisenberg(N)
    assert np.linalg.norm(H @ psi - E * psi) < 1e-9


def test_heisenberg_ground_state_sector_and_mps():
    N = 10
    psi, E = W.heisenberg_ground_state(N)
    idx = np.arange(2 ** N)
    pop = np.array([bin(i).count("1") for i in idx])
    assert np.all(psi[pop != N // 2] == 0.0)       # total S^z = 0
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-14
    # with chi = 2^(N/2) the compression is exact
    A = W.heisenberg_mps(N, chi=32)
    v = mps.to_dense(A)
    # to_dense puts site 0 first (most significant); psi has qubit j at bit j
    t = psi.reshape((2,) * N).transpose(tuple(range(N - 1, -1, -1))).reshape(-1)
    assert abs(abs(np.vdot(t, v)) - 1.0) < 1e-12
    for j in range(1, N):
        assert mps.is_right_isometric(A[j])
    # a smaller chi truncates: still unit norm, overlap close to one
    B = W.heisenberg_mps(N, chi=8)
    assert max(a.shape[2] for a in B) == 8
    assert abs(mps.norm(B) - 1.0) < 1e-12
    assert abs(mps.overlap(B, A)) > 0.99


def test_serving_mix_follows_the_recipe():
    specs = W.serving_mix(200, seed=4)
    assert {s["task"] for s in specs} == {"x", "cnot", "ghz", "heisenberg"}
    for s in specs:
        assert s["N"] in (10, 20, 30, 50) and s["chi"] in (16, 32, 64, 128)
        assert s["K"] in (8, 32, 128) and 100 <= s["M"] <= 300
        assert s["R"] == (4 if s["task"] in ("x", "cnot") else 1)
        if s["task"] == "heisenberg":
            assert s["N"] == 20
    assert W.serving_mix(5, seed=4) == specs[:5]
