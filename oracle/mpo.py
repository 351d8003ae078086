"""Gate objective with matrix-product operators (oracle; test infrastructure
only).

The paper's figure of merit for gates (Sec. II, Eqs. 5-6): the propagator
U(T) is evolved as an MPO from the identity by the same Trotter slices as the
states, compressed by truncated SVDs after every step, and scored by

    F = 1/K sum_k |tr(U_T^dag U_k(T)) / 2^n|^2.

Representation: site j of an operator is an array (D_j, 4, D_{j+1}) whose
physical index p = 2 s + t pairs the output index s and the input index t of
qubit j, and the list holds vec(U) / 2^{n/2}, the operator as a vector of
unit norm (the identity is the product of vec(I_2) / sqrt 2).  A gate G
acting on U from the left acts on that vector as G (x) I on each p, the
overlap of two such vectors is tr(A^dag B) / 2^n, and TEBD on the vectors
(oracle/tebd.py's sweep, split and truncation rule with d = 4) is TEBD on the
MPO: the same SVD of the two-site tensor, the same kept singular values.

The gradient is the adjoint of oracle/grape.py on these vectors: the
costate is vec(U_T) propagated backward, and every insertion G acts as
G (x) I (App. A for the propagated operators).  The sweep order, the
first-order split and the Heisenberg crosstalk with its mid-sweep u^zz
insertions are those of the state path.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import gates, grape, tebd
from .mps import MPS, copy, overlap, right_canonicalize

I2 = np.eye(2, dtype=np.complex128)
ZOUT = np.repeat(gates.ZVALS, 2)          # Z on the output index of p = 2 s + t


def embed(G: np.ndarray) -> np.ndarray:
    """2x2 operator on the output index -> 4x4 on p (G (x) I)."""
    return np.kron(G, I2)


def embed_bond(G: np.ndarray) -> np.ndarray:
    """(2, 2, 2, 2) two-qubit gate [s1, s2, u1, u2] -> (4, 4, 4, 4) on
    (p1, p2, q1, q2), identity on the input indices."""
    return np.einsum("abcd,ef,gh->aebgcfdh", G, I2, I2).reshape(4, 4, 4, 4)


def operator_product(mats) -> MPS:
    """Bond-1 MPO of the tensor product of single-qubit operators, each factor
    divided by sqrt 2 (so a product of unitaries is a unit vector)."""
    return [(np.asarray(m, np.complex128) / np.sqrt(2.0)).reshape(1, 4, 1) for m in mats]


def identity(n: int) -> MPS:
    return operator_product([I2] * n)


def cnot_pair() -> MPS:
    """CNOT (control first) = |0><0| (x) I + |1><1| (x) X as a bond-2 MPO."""
    P0 = np.diag([1.0, 0.0]).astype(np.complex128)
    P1 = np.diag([0.0, 1.0]).astype(np.complex128)
    left = np.stack([P0.reshape(4), P1.reshape(4)], axis=1).reshape(1, 4, 2) / np.sqrt(2.0)
    right = np.stack([I2.reshape(4), gates.X.reshape(4)], axis=0).reshape(2, 4, 1) / np.sqrt(2.0)
    return [left, right]


def gate_target(task: str, n: int) -> MPS:
    """U_T of the gate tasks of Sec. III: the parallel X gate, or CNOT on the
    pairs (2p, 2p+1) (a last unpaired qubit gets the identity)."""
    if task == "x":
        return operator_product([gates.X] * n)
    if task == "cnot":
        out: MPS = []
        for _ in range(n // 2):
            out += cnot_pair()
        if n % 2:
            out += identity(1)
        return out
    raise ValueError(f"gate objective for the gate tasks only, not {task!r}")


def to_matrix(W: MPS) -> np.ndarray:
    """The 2^n x 2^n operator (the stored vector times 2^{n/2}); qubit 0 is the
    most significant index of rows (outputs) and columns (inputs)."""
    n = len(W)
    v = np.ones((1, 1), np.complex128)
    for A in W:
        Dl, d, Dr = A.shape
        v = (v @ A.reshape(Dl, d * Dr)).reshape(-1, Dr)
    t = v[:, 0].reshape((2, 2) * n)                 # (s0, t0, s1, t1, ...)
    t = t.transpose(tuple(range(0, 2 * n, 2)) + tuple(range(1, 2 * n, 2)))
    return t.reshape(2 ** n, 2 ** n) * 2.0 ** (n / 2)


def _bond_gate_fn(problem, k: int, l: int, adjoint: bool):
    if gates.heisenberg(problem):
        G = [embed_bond(g) for g in gates.bond_gates(problem, k, l)]
        if adjoint:
            G = [np.conj(np.transpose(g, (2, 3, 0, 1))) for g in G]
        return lambda b, th: np.einsum("stuv,auvc->astc", G[b], th)
    phis = problem.dt * gates.couplings(problem, k)[l]
    sign = -1.0 if adjoint else 1.0
    ph = [np.exp(-1j * sign * phis[b] * np.outer(ZOUT, ZOUT)) for b in range(problem.N - 1)]
    return lambda b, th: th * ph[b][None, :, :, None]


def _layer(G2s) -> np.ndarray:
    return np.array([embed(g) for g in G2s])


def forward_slice(problem, W: MPS, l: int, k: int, chi: Optional[int] = None, stats=None,
                  after=None) -> MPS:
    """U <- U_l U (0-based l), as oracle/tebd.py's forward slice."""
    chi = problem.chi if chi is None else chi
    a = tebd.rotation_layer(W, _layer(gates.slice_pre(problem, l)))
    a = tebd.bond_sweep(a, _bond_gate_fn(problem, k, l, False), tebd.forward_ltr(problem, l),
                        chi, problem.eps, problem.renormalize, stats, after=after)
    return tebd.rotation_layer(a, _layer(gates.slice_post(problem, l)))


def backward_slice(problem, B: MPS, l: int, k: int, chi: Optional[int] = None, stats=None,
                   before=None) -> MPS:
    """B <- U_l^dag B (0-based l)."""
    chi = problem.chi if chi is None else chi
    dag = lambda G: np.conj(np.transpose(G, (0, 2, 1)))
    b = tebd.rotation_layer(B, _layer(dag(gates.slice_post(problem, l))))
    b = tebd.bond_sweep(b, _bond_gate_fn(problem, k, l, True), not tebd.forward_ltr(problem, l),
                        chi, problem.eps, problem.renormalize, stats, before=before)
    return tebd.rotation_layer(b, _layer(dag(gates.slice_pre(problem, l))))


def evolve(problem, k: int, chi: Optional[int] = None, keep_all: bool = False, stats=None):
    """U_k(T) (or every U after 0..M slices) from the identity."""
    cur = identity(problem.N)
    states = [cur]
    for l in range(problem.M):
        cur = forward_slice(problem, cur, l, k, chi, stats)
        states.append(cur)
    return states if keep_all else cur


def _insertions(problem, bra: MPS, ket: MPS, l: int, dux, duy, duzz):
    """The boundary insertions of oracle/grape.py at boundary l (1-based), each
    operator embedded as G (x) I."""
    N, M, dt = problem.N, problem.M, problem.dt
    E, F = grape.environments(bra, ket)
    rho = grape.transitions(bra, ket, E, F)
    if l >= 1:
        s = l - 1
        post = gates.slice_post(problem, s)
        for j in range(N):
            _, P, _, (dx, dy) = gates.site_factors(problem, s, j)
            dux[s, j] += np.sum(embed(dx @ P.conj().T) * rho[j])
            duy[s, j] += np.sum(embed(dy @ P.conj().T) * rho[j])
        if not gates.heisenberg(problem):
            for b in range(N - 1):
                if not problem.zz_mask[b]:
                    continue
                W1 = embed(post[b] @ gates.Z @ post[b].conj().T)
                W2 = embed(post[b + 1] @ gates.Z @ post[b + 1].conj().T)
                duzz[s, b] += -1j * dt * grape.two_site_element(bra, ket, E, F, b, W1, W2)
    if l <= M - 1 and gates.order(problem) == 2:
        s = l
        for j in range(N):
            Q, _, (dx, dy), _ = gates.site_factors(problem, s, j)
            dux[s, j] += np.sum(embed(Q.conj().T @ dx) * rho[j])
            duy[s, j] += np.sum(embed(Q.conj().T @ dy) * rho[j])


def _zz_out(state: MPS, b: int) -> MPS:
    out = copy(state)
    out[b] = out[b] * ZOUT[None, :, None]
    out[b + 1] = out[b + 1] * ZOUT[None, :, None]
    return out


def sample_grad(problem, k: int, target: MPS, chi: Optional[int] = None):
    """O_k = tr(U_T^dag U_k) / 2^n and dO_k/du for noise sample k.
    Returns (O, dux (M, N), duy (M, N), duzz (M, N-1))."""
    N, M = problem.N, problem.M
    a = evolve(problem, k, chi, keep_all=True)
    O = overlap(target, a[M])
    b = right_canonicalize(target)
    dux = np.zeros((M, N), np.complex128)
    duy = np.zeros((M, N), np.complex128)
    duzz = np.zeros((M, N - 1), np.complex128)
    mid = gates.heisenberg(problem) and problem.zz_mask.any()
    for l in range(M, -1, -1):
        _insertions(problem, b, a[l], l, dux, duy, duzz)
        if l >= 1:
            s = l - 1
            if mid:
                alpha = {}
                forward_slice(problem, a[s], s, k, chi,
                              after=lambda bd, st: alpha.__setitem__(bd, copy(st)))

                def before(bd, st, s=s, alpha=alpha):
                    if problem.zz_mask[bd]:
                        duzz[s, bd] += -1j * problem.dt * overlap(st, _zz_out(alpha[bd], bd))
                b = backward_slice(problem, b, s, k, chi, before=before)
            else:
                b = backward_slice(problem, b, s, k, chi)
    return O, dux, duy, duzz


def gate_fidelity_grad(problem, target: Optional[MPS] = None, chi: Optional[int] = None):
    """F = 1/K sum_k |tr(U_T^dag U_k(T))/2^n|^2 and dF/du (float64, the control
    layout of oracle/grape.py).  The target defaults to the task's gate."""
    target = gate_target(problem.task, problem.N) if target is None else target
    N, M, K = problem.N, problem.M, problem.K
    F = 0.0
    gux = np.zeros((M, N))
    guy = np.zeros((M, N))
    guzz = np.zeros((M, N - 1))
    overlaps = []
    for k in range(K):
        O, dux, duy, duzz = sample_grad(problem, k, target, chi)
        overlaps.append(O)
        F += abs(O) ** 2
        gux += 2.0 * np.real(np.conj(O) * dux)
        guy += 2.0 * np.real(np.conj(O) * duy)
        guzz += 2.0 * np.real(np.conj(O) * duzz)
    return dict(F=F / K, g_ux=gux / K, g_uy=guy / K, g_uzz=guzz / K, overlaps=overlaps)
