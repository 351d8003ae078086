"""Gates of one Trotter slice (oracle; test infrastructure only).

Drive term per site: h = (u^x X + u^y Y) / 2 (Sec. III, Eq. 8 in the
normalisation of the workloads, with the 1/2 on the drive).  A slice of
length dt is split second-order as U = R Z R (Strang), where

    R = exp(-i (dt/2) h)   on every site,
    Z = exp(-i dt sum_b c_b Z_b Z_{b+1})   (all ZZ terms commute, so exact),

the rightmost factor acting first.  The paper's Eq. 4 is the first-order
product of the same three kinds of factor, U = X Y Z with

    X = exp(-i dt u^x X / 2),   Y = exp(-i dt u^y Y / 2)   on every site;

``problem.order`` (2, the default, or 1) selects the split.  Either way a
slice is U = post . Z . pre with per-site 2x2 factors: pre = post = R
(second order) or pre = I, post = X Y (first order).

With the paper's Heisenberg-type crosstalk (Sec. III, Eq. 9) the two-site
factor of bond b is the 4x4 exponential

    G_b = exp(-i dt (J^x XX + J^y YY + c_b ZZ)),   c_b = u^zz + J^z,

and Z is the ordered product of the G_b over the bonds in the order the
slice's sweep visits them (the terms of neighbouring bonds do not commute;
oracle/tebd.py fixes the order).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ZVALS = np.array([1.0, -1.0])  # eigenvalue of Z on |0>, |1>


def _f(a: float, r: float) -> float:
    """sin(a r) / r, continuous at r = 0."""
    return a * np.sinc(a * r / np.pi)


def _g(a: float, r: float) -> float:
    """f'(r) / r = (a r cos(a r) - sin(a r)) / r^3, by series near r = 0."""
    x = a * r
    if x < 0.1:
        x2 = x * x
        # sum_{n>=1} (-1)^n (2n)/(2n+1)! x^(2n-2)
        return a ** 3 * (-1.0 / 3.0 + x2 / 30.0 - x2 * x2 / 840.0
                         + x2 ** 3 / 45360.0 - x2 ** 4 / 3991680.0)
    return (x * np.cos(x) - np.sin(x)) / r ** 3


def half_rotation(ux: float, uy: float, dt: float) -> np.ndarray:
    """R = exp(-i (dt/2) (ux X + uy Y)/2) = cos(a r) I - i sin(a r)/r (ux X + uy Y).

    a = dt/4, r = sqrt(ux^2 + uy^2).
    """
    a = dt / 4.0
    r = float(np.hypot(ux, uy))
    return np.cos(a * r) * I2 - 1j * _f(a, r) * (ux * X + uy * Y)


def half_rotation_derivs(ux: float, uy: float, dt: float):
    """(dR/dux, dR/duy) of ``half_rotation`` in closed form."""
    a = dt / 4.0
    r = float(np.hypot(ux, uy))
    f = _f(a, r)
    g = _g(a, r)
    n = ux * X + uy * Y
    dx = -a * ux * f * I2 - 1j * (g * ux * n + f * X)
    dy = -a * uy * f * I2 - 1j * (g * uy * n + f * Y)
    return dx, dy


def zz_phase(phi: float) -> np.ndarray:
    """exp(-i phi Z x Z) as a 2x2 array over (s, s'): exp(-i phi z_s z_s')."""
    return np.exp(-1j * phi * np.outer(ZVALS, ZVALS))


def heisenberg(problem) -> bool:
    return getattr(problem, "xt_model", "zz") == "heisenberg"


def couplings(problem, k: int) -> np.ndarray:
    """ZZ coefficient c[l, b] = zz_mask_b u^zz[l, b] + xt_mask_b J^z[k, b],
    shape (M, N-1) (J^z is J[k, b] in the ZZ model)."""
    Jz = problem.J[k][:, 2] if heisenberg(problem) else problem.J[k]
    return (problem.zz_mask[None, :] * problem.uzz
            + problem.xt_mask[None, :] * Jz[None, :])


XX = np.kron(X, X)
YY = np.kron(Y, Y)
ZZ = np.kron(Z, Z)


def bond_hamiltonian(jx: float, jy: float, cz: float) -> np.ndarray:
    """jx XX + jy YY + cz ZZ, 4x4 over (s_b, s_{b+1}) with s_b the major index."""
    return jx * XX + jy * YY + cz * ZZ


def bond_gate(jx: float, jy: float, cz: float, dt: float) -> np.ndarray:
    """exp(-i dt (jx XX + jy YY + cz ZZ)) as a (2, 2, 2, 2) array
    [s, t, s', t'] (out site b, out site b+1, in site b, in site b+1)."""
    return scipy.linalg.expm(-1j * dt * bond_hamiltonian(jx, jy, cz)).reshape(2, 2, 2, 2)


def bond_gates(problem, k: int, l: int):
    """G_b of slice l (0-based), noise sample k, for every bond (Heisenberg
    crosstalk model)."""
    c = couplings(problem, k)[l]
    J = problem.J[k]
    xm = problem.xt_mask
    return [bond_gate(xm[b] * J[b, 0], xm[b] * J[b, 1], c[b], problem.dt)
            for b in range(problem.N - 1)]


def slice_rotations(problem, l: int) -> np.ndarray:
    """R[j] for slice l (0-based), shape (N, 2, 2)."""
    return np.array([half_rotation(problem.ux[l, j], problem.uy[l, j],
                                   problem.dt) for j in range(problem.N)])


def first_order_rotation(ux: float, uy: float, dt: float) -> np.ndarray:
    """G = exp(-i dt ux X/2) exp(-i dt uy Y/2) (the X and Y layers of Eq. 4)."""
    cx, sx = np.cos(dt * ux / 2.0), np.sin(dt * ux / 2.0)
    cy, sy = np.cos(dt * uy / 2.0), np.sin(dt * uy / 2.0)
    return (cx * I2 - 1j * sx * X) @ (cy * I2 - 1j * sy * Y)


def first_order_rotation_derivs(ux: float, uy: float, dt: float):
    """(dG/dux, dG/duy): (-i dt/2 X) G and exp(-i dt ux X/2) (-i dt/2 Y) exp(-i dt uy Y/2)."""
    cx, sx = np.cos(dt * ux / 2.0), np.sin(dt * ux / 2.0)
    cy, sy = np.cos(dt * uy / 2.0), np.sin(dt * uy / 2.0)
    Xr = cx * I2 - 1j * sx * X
    Yr = cy * I2 - 1j * sy * Y
    return (-0.5j * dt) * X @ Xr @ Yr, Xr @ ((-0.5j * dt) * Y) @ Yr


def order(problem) -> int:
    return int(getattr(problem, "order", 2))


def site_factors(problem, l: int, j: int):
    """(pre, post, dpre, dpost) of site j in slice l (0-based); dpre and dpost
    are (d/dux, d/duy) pairs, dpre None where pre does not depend on u."""
    ux, uy, dt = problem.ux[l, j], problem.uy[l, j], problem.dt
    if order(problem) == 1:
        return I2, first_order_rotation(ux, uy, dt), None, first_order_rotation_derivs(ux, uy, dt)
    R = half_rotation(ux, uy, dt)
    d = half_rotation_derivs(ux, uy, dt)
    return R, R, d, d


def slice_pre(problem, l: int) -> np.ndarray:
    """pre[j] of slice l, shape (N, 2, 2)."""
    return np.array([site_factors(problem, l, j)[0] for j in range(problem.N)])


def slice_post(problem, l: int) -> np.ndarray:
    """post[j] of slice l, shape (N, 2, 2)."""
    return np.array([site_factors(problem, l, j)[1] for j in range(problem.N)])
