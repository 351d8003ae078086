"""Ensemble fidelity and its exact adjoint gradient (oracle; test infrastructure only).

Objective (Sec. II, Eq. 7, scored on R product-state inputs per noise sample):

    F = 1/(K R) sum_{k,r} |O_kr|^2,      O_kr = <T_r | a_M^{(k,r)}>

Adjoint (App. A, Eqs. A1-A2): with a_l the forward state after slice l and
b_{l+1} the target propagated backward through slices M..l+1, every derivative
of O is a matrix element <b_{l+1}| G |a_l> of a local operator G placed where
the control enters.  For the second-order slice U_l = R_l Z_l R_l:

  * left (outer) half rotation of slice l:   G = dR_{l,j} R_{l,j}^dagger   at site j
  * right (inner) half rotation of slice l+1: G = R_{l+1,j}^dagger dR_{l+1,j} at site j
  * ZZ control of slice l on bond b:
        G = -i dt (R_{l,b} Z R_{l,b}^dagger) (x) (R_{l,b+1} Z R_{l,b+1}^dagger)

For the paper's first-order split U_l = X_l Y_l Z_l only the outer factor
P = X_l Y_l depends on the drive: G = dP P^dagger (that is -i dt/2 X and
X_l (-i dt/2 Y) X_l^dagger, the insertions of App. A with their -i dt
factor) and the ZZ insertion uses P in place of R.

(the paper's Eq. A2 shows the first-order form without the -i dt factor; the
factor and the positions follow from differentiating the slice).  All matrix
elements at one boundary come from one pass of left/right transfer
environments.  dF = 1/(K R) sum 2 Re(conj(O_kr) dO_kr), with the final forward
overlap O_kr for every boundary.

With Heisenberg crosstalk the bond gates of one slice do not commute, so
Z Z_b cannot be moved to the slice boundary.  For the sweep order of
oracle/tebd.py (bond b visited after the bonds before it in the sweep),
d/du^zz_b of the ordered product is the product with -i dt Z_b Z_{b+1}
placed right after G_b (Z Z commutes with its own bond gate), and its matrix
element is

    -i dt <beta_b | Z_b Z_{b+1} | alpha_b>,

alpha_b the forward working state of the two-site layer just after bond b is
updated, beta_b the backward working state of the same slice just before
bond b is updated (the backward slice undoes the bonds in the opposite
order, so beta_b has undone exactly the gates that follow G_b).  Both are the
truncated states the two sweeps produce.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import gates, tebd
from .mps import MPS, copy, overlap, product_state, right_canonicalize


def environments(bra: MPS, ket: MPS):
    """Left E[0..N] and right F[0..N] transfer environments of <bra|ket>."""
    N = len(ket)
    E = [None] * (N + 1)
    F = [None] * (N + 1)
    d = ket[0].shape[1]
    E[0] = np.ones((1, 1), np.complex128)
    for j in range(N):
        E[j + 1] = sum(bra[j][:, s, :].conj().T @ E[j] @ ket[j][:, s, :]
                       for s in range(d))
    F[N] = np.ones((1, 1), np.complex128)
    for j in range(N - 1, -1, -1):
        F[j] = sum(ket[j][:, s, :] @ F[j + 1] @ bra[j][:, s, :].conj().T
                   for s in range(d))
    return E, F


def transitions(bra: MPS, ket: MPS, E, F) -> np.ndarray:
    """rho[j, s, s'] = <bra| (|s><s'|)_j |ket>, shape (N, d, d)."""
    N = len(ket)
    d = ket[0].shape[1]
    rho = np.zeros((N, d, d), np.complex128)
    for j in range(N):
        for s in range(d):
            for t in range(d):
                rho[j, s, t] = np.trace(bra[j][:, s, :].conj().T @ E[j]
                                        @ ket[j][:, t, :] @ F[j + 1])
    return rho


def two_site_element(bra: MPS, ket: MPS, E, F, b: int, G1: np.ndarray,
                     G2: np.ndarray) -> complex:
    """<bra| (G1)_b (G2)_{b+1} |ket>."""
    val = 0.0 + 0.0j
    d = ket[0].shape[1]
    for s1 in range(d):
        for t1 in range(d):
            if G1[s1, t1] == 0:
                continue
            W = bra[b][:, s1, :].conj().T @ E[b] @ ket[b][:, t1, :]
            for s2 in range(d):
                for t2 in range(d):
                    if G2[s2, t2] == 0:
                        continue
                    val += G1[s1, t1] * G2[s2, t2] * np.trace(
                        bra[b + 1][:, s2, :].conj().T @ W
                        @ ket[b + 1][:, t2, :] @ F[b + 2])
    return complex(val)


def boundary_insertions(problem, bra: MPS, ket: MPS, l: int, dux, duy, duzz):
    """Accumulate every dO contribution at boundary l (1-based, 0..M):
    pair (b_{l+1}, a_l).  Slice s is U_s = post Z pre (oracle/gates.py)."""
    N, M, dt = problem.N, problem.M, problem.dt
    E, F = environments(bra, ket)
    rho = transitions(bra, ket, E, F)
    if l >= 1:                                   # outer factor of slice l
        s = l - 1
        post = gates.slice_post(problem, s)
        for j in range(N):
            _, P, _, (dx, dy) = gates.site_factors(problem, s, j)
            dux[s, j] += np.sum((dx @ P.conj().T) * rho[j])
            duy[s, j] += np.sum((dy @ P.conj().T) * rho[j])
        for b in range(N - 1):
            if not problem.zz_mask[b] or gates.heisenberg(problem):
                continue
            W1 = post[b] @ gates.Z @ post[b].conj().T
            W2 = post[b + 1] @ gates.Z @ post[b + 1].conj().T
            duzz[s, b] += -1j * dt * two_site_element(bra, ket, E, F, b, W1, W2)
    if l <= M - 1 and gates.order(problem) == 2:  # inner factor of slice l+1
        s = l
        for j in range(N):
            Q, _, (dx, dy), _ = gates.site_factors(problem, s, j)
            dux[s, j] += np.sum((Q.conj().T @ dx) * rho[j])
            duy[s, j] += np.sum((Q.conj().T @ dy) * rho[j])


def trajectory(problem, k: int, r: int, chi: Optional[int] = None,
               stats=None):
    """O_kr and dO_kr/du for one trajectory.

    Returns (O, dux (M,N), duy (M,N), duzz (M,N-1)), all complex.
    """
    N, M = problem.N, problem.M
    a = tebd.evolve(problem, product_state(problem.inputs[r]), k,
                    keep_all=True, chi=chi, stats=stats)
    T = problem.targets[r]
    O = overlap(T, a[M])
    b = right_canonicalize(T)
    dux = np.zeros((M, N), np.complex128)
    duy = np.zeros((M, N), np.complex128)
    duzz = np.zeros((M, N - 1), np.complex128)
    for l in range(M, -1, -1):
        boundary_insertions(problem, b, a[l], l, dux, duy, duzz)
        if l >= 1:
            if gates.heisenberg(problem) and problem.zz_mask.any():
                b = _backward_with_zz(problem, a[l - 1], b, l - 1, k, chi, stats, duzz)
            else:
                b = tebd.backward_slice(problem, b, l - 1, k, chi, stats)
    return O, dux, duy, duzz


def _zz_on_bond(state: MPS, b: int) -> MPS:
    out = copy(state)
    out[b] = out[b] * gates.ZVALS[None, :, None]
    out[b + 1] = out[b + 1] * gates.ZVALS[None, :, None]
    return out


def _backward_with_zz(problem, a_prev: MPS, b_next: MPS, s: int, k: int, chi, stats, duzz):
    """Backward slice s with the mid-sweep u^zz insertions (Heisenberg
    crosstalk): alpha_b from re-running forward slice s on a_{s}, beta_b from
    the backward sweep itself."""
    alpha = {}
    tebd.forward_slice(problem, a_prev, s, k, chi,
                       after=lambda bd, st: alpha.__setitem__(bd, copy(st)))

    def before(bd, st):
        if problem.zz_mask[bd]:
            duzz[s, bd] += -1j * problem.dt * overlap(st, _zz_on_bond(alpha[bd], bd))
    return tebd.backward_slice(problem, b_next, s, k, chi, stats, before=before)


def fidelity_grad(problem, chi: Optional[int] = None, trajectories=None,
                  details: bool = False):
    """F and dF/du over the ensemble (or over the listed (k, r) trajectories).

    Returns a dict with F, g_ux, g_uy, g_uzz (float64, control layout) and the
    overlaps O[k, r]; with ``details`` also the per-trajectory dO arrays.
    """
    N, M = problem.N, problem.M
    if trajectories is None:
        trajectories = [(k, r) for k in range(problem.K) for r in range(problem.R)]
    n = len(trajectories)
    F = 0.0
    gux = np.zeros((M, N))
    guy = np.zeros((M, N))
    guzz = np.zeros((M, N - 1))
    O_all = {}
    per = {}
    for (k, r) in trajectories:
        O, dux, duy, duzz = trajectory(problem, k, r, chi)
        O_all[(k, r)] = O
        F += abs(O) ** 2
        gux += 2.0 * np.real(np.conj(O) * dux)
        guy += 2.0 * np.real(np.conj(O) * duy)
        guzz += 2.0 * np.real(np.conj(O) * duzz)
        if details:
            per[(k, r)] = (dux, duy, duzz)
    out = dict(F=F / n, g_ux=gux / n, g_uy=guy / n, g_uzz=guzz / n,
               overlaps=O_all)
    if details:
        out["dO"] = per
    return out


def final_states(problem, chi: Optional[int] = None):
    """a_M for every trajectory t = k R + r (list of MPS)."""
    out = []
    for k in range(problem.K):
        for r in range(problem.R):
            out.append(tebd.evolve(problem, product_state(problem.inputs[r]),
                                   k, chi=chi))
    return out
