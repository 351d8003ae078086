"""Host logic of the sequential optimisation (Sec. II; no GPU needed): the
error-strength steps, the control extension that seeds n qubits from a
smaller solution, and the parasitic-term count that sizes the two-stage
ensemble."""
import os

import numpy as np
import pytest
import torch

import workloads as W


@pytest.fixture(scope="module")
def O():
    from conftest import ensure_library
    ensure_library()
    from paper_2603_03639_amd import optimize
    return optimize


def test_robustness_steps(O):
    assert O.robustness_steps(0.05) == pytest.approx([0.0, 0.01, 0.02, 0.03, 0.04, 0.05])
    assert O.robustness_steps(0.0) == [0.0]
    with pytest.raises(ValueError):
        O.robustness_steps(0.025)


def test_extend_controls_keeps_old_qubits_and_continues_the_pattern(O):
    rng = np.random.default_rng(3)
    M, n = 5, 4
    ux, uy = rng.standard_normal((M, n)), rng.standard_normal((M, n))
    uzz = np.zeros((M, n - 1))
    uzz[:, 0::2] = rng.standard_normal((M, 2))          # pair bonds 0, 2
    a, b, c = O.extend_controls(ux, uy, uzz, 7)
    assert a.shape == (M, 7) and b.shape == (M, 7) and c.shape == (M, 6)
    assert np.array_equal(a[:, :n].numpy(), ux) and np.array_equal(c[:, :n - 1].numpy(), uzz)
    # added qubits repeat the qubit two places before, added bonds likewise
    for j in range(n, 7):
        assert np.array_equal(a[:, j].numpy(), a[:, j - 2].numpy())
        assert np.array_equal(b[:, j].numpy(), b[:, j - 2].numpy())
    for bnd in range(n - 1, 6):
        assert np.array_equal(c[:, bnd].numpy(), c[:, bnd - 2].numpy())
    # the CNOT pair pattern (u^zz on even bonds only) survives
    assert np.all(c[:, 1::2].numpy() == 0.0) and np.all(c[:, 4].numpy() == uzz[:, 2])
    with pytest.raises(ValueError):
        O.extend_controls(ux, uy, uzz, 3)


def test_parasitic_count(O):
    from paper_2603_03639_amd import tnrg
    pz = W.make_problem(task="cnot", N=10, M=2, K=1, R=1)
    ph = W.make_problem(task="cnot", N=10, M=2, K=1, R=1, xt_model="heisenberg")
    # ZZ model of the CNOT task: crosstalk on the 4 bonds between pairs;
    # Heisenberg: three strengths on each of the 9 bonds
    assert O.parasitic_count(tnrg.Model.from_problem(pz)) == 4
    assert O.parasitic_count(tnrg.Model.from_problem(ph)) == 27


def test_bucket_sequence_floor(O):
    """The capacity search never tries a bucket below the largest bond of the
    inputs and targets, even where chi is smaller (the states hold them
    before their first truncation to chi)."""
    from paper_2603_03639_amd import tnrg
    m = lambda N, chi: tnrg.Model(N=N, M=1, dt=0.1, chi=chi)
    assert tnrg._bucket_sequence(m(50, 64), None) == [4, 8, 16, 32, 64]
    assert tnrg._bucket_sequence(m(50, 64), None, floor=5) == [8, 16, 32, 64]
    assert tnrg._bucket_sequence(m(8, 1), None) == [1]
    assert tnrg._bucket_sequence(m(8, 1), None, floor=2) == [2]
    assert tnrg._bucket_sequence(m(50, 64), 16, floor=2) == [16, 32, 64]
