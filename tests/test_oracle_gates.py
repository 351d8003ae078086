"""Pins of the oracle's single-slice gates against library routines.

The half rotation is checked against scipy's matrix exponential of its
generator, its derivative against scipy's Frechet derivative of expm and
against central differences, the ZZ phase against the exponential of the
4x4 diagonal generator.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import gates

X = np.array([[0, 1], [1, 0]], complex)
Y = np.array([[0, -1j], [1j, 0]], complex)
Z = np.diag([1.0, -1.0]).astype(complex)

CASES = [(0.3, -0.7, 0.2), (1.0, 1.0, 0.05), (0.0, 0.0, 0.2), (1e-9, 2e-9, 0.1),
         (-0.9, 0.0, 0.3), (0.0, 0.6, 0.01), (5.0, -3.0, 0.2), (1e-4, -1e-4, 0.5)]


@pytest.mark.parametrize("ux,uy,dt", CASES)
def test_half_rotation_is_expm(ux, uy, dt):
    gen = -1j * (dt / 2) * (ux * X + uy * Y) / 2
    ref = scipy.linalg.expm(gen)
    assert np.abs(gates.half_rotation(ux, uy, dt) - ref).max() < 1e-14


@pytest.mark.parametrize("ux,uy,dt", CASES)
def test_half_rotation_derivative_is_frechet(ux, uy, dt):
    dx, dy = gates.half_rotation_derivs(ux, uy, dt)
    gen = -1j * (dt / 2) * (ux * X + uy * Y) / 2
    _, fx = scipy.linalg.expm_frechet(gen, -1j * (dt / 2) * X / 2)
    _, fy = scipy.linalg.expm_frechet(gen, -1j * (dt / 2) * Y / 2)
    assert np.abs(dx - fx).max() < 1e-13
    assert np.abs(dy - fy).max() < 1e-13


@pytest.mark.parametrize("ux,uy,dt", CASES[:4])
def test_half_rotation_derivative_central_difference(ux, uy, dt):
    h = 1e-6
    dx, dy = gates.half_rotation_derivs(ux, uy, dt)
    fdx = (gates.half_rotation(ux + h, uy, dt) - gates.half_rotation(ux - h, uy, dt)) / (2 * h)
    fdy = (gates.half_rotation(ux, uy + h, dt) - gates.half_rotation(ux, uy - h, dt)) / (2 * h)
    assert np.abs(dx - fdx).max() < 1e-9
    assert np.abs(dy - fdy).max() < 1e-9


def test_half_rotation_unitary_and_composes_to_pi_pulse():
    T, M = 10.0, 50
    R = gates.half_rotation(np.pi / T, 0.0, T / M)
    assert np.abs(R @ R.conj().T - np.eye(2)).max() < 1e-15
    # 2M half slices of the global pi pulse give exp(-i pi X / 2) = -i X
    # (Sec. III: a global pi pulse along X realises the parallel X gate).
    U = np.linalg.matrix_power(R, 2 * M)
    assert np.abs(U - (-1j) * X).max() < 1e-13


@pytest.mark.parametrize("phi", [0.0, 0.013, -0.7, 2.5])
def test_zz_phase(phi):
    ref = scipy.linalg.expm(-1j * phi * np.kron(Z, Z))
    got = gates.zz_phase(phi).reshape(4)
    assert np.abs(np.diag(ref) - got).max() < 1e-15
    assert np.abs(ref - np.diag(np.diag(ref))).max() == 0.0
