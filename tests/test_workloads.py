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
