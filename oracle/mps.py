"""Matrix-product states (oracle; test infrastructure only).

An MPS is a list of N complex128 arrays A[j] of shape (D_j, d, D_{j+1}) with
D_0 = D_N = 1, the state being
    psi(s_0 .. s_{N-1}) = A[0][:, s_0, :] A[1][:, s_1, :] ... A[N-1][:, s_{N-1}, :]
(the first and last factors are row and column vectors, Sec. II).
"""
from __future__ import annotations

from typing import List

import numpy as np

MPS = List[np.ndarray]


def product_state(vecs) -> MPS:
    """Bond-1 MPS of the product state  (x)_j vecs[j]  (Sec. IV initial state)."""
    return [np.asarray(v, np.complex128).reshape(1, 2, 1).copy() for v in vecs]


def copy(mps: MPS) -> MPS:
    return [a.copy() for a in mps]


def bond_dims(mps: MPS) -> List[int]:
    return [mps[0].shape[0]] + [a.shape[2] for a in mps]


def overlap(bra: MPS, ket: MPS) -> complex:
    """<bra|ket>, conjugate-linear in ``bra``, by left transfer matrices.

    E_0 = 1,  E_{j+1} = sum_s B_j[s]^dagger E_j A_j[s],  result E_N.
    """
    E = np.ones((1, 1), np.complex128)
    for B, A in zip(bra, ket):
        E = sum(B[:, s, :].conj().T @ E @ A[:, s, :] for s in range(A.shape[1]))
    return complex(E[0, 0])


def norm(mps: MPS) -> float:
    return float(np.sqrt(abs(overlap(mps, mps))))


def to_dense(mps: MPS) -> np.ndarray:
    """State vector, site 0 being the most significant qubit."""
    v = np.ones((1, 1), np.complex128)  # (amplitude index, right bond)
    for A in mps:
        Dl, d, Dr = A.shape
        v = (v @ A.reshape(Dl, d * Dr)).reshape(-1, Dr)
    return v[:, 0].copy()


def right_canonicalize(mps: MPS) -> MPS:
    """QR sweep right to left: sites 1..N-1 right-isometric, norm moved to
    site 0, which is then normalised to 1."""
    out = copy(mps)
    for j in range(len(out) - 1, 0, -1):
        A = out[j]
        Dl, d, Dr = A.shape
        # A = L Q with orthonormal rows of Q: QR of A^dagger.
        q, r = np.linalg.qr(A.reshape(Dl, d * Dr).conj().T)
        k = q.shape[1]
        out[j] = q.conj().T.reshape(k, d, Dr)
        L = r.conj().T                      # (Dl, k)
        P = out[j - 1]
        out[j - 1] = np.einsum("asb,bc->asc", P, L)
    out[0] = out[0] / np.linalg.norm(out[0])
    return out


def is_right_isometric(A: np.ndarray, tol: float = 1e-12) -> bool:
    Dl = A.shape[0]
    m = A.reshape(Dl, -1)
    return bool(np.allclose(m @ m.conj().T, np.eye(Dl), atol=tol))


def is_left_isometric(A: np.ndarray, tol: float = 1e-12) -> bool:
    Dr = A.shape[2]
    m = A.reshape(-1, Dr)
    return bool(np.allclose(m.conj().T @ m, np.eye(Dr), atol=tol))


def apply_site(mps: MPS, j: int, G: np.ndarray) -> MPS:
    """(G)_j |mps>: A_j[:, s, :] <- sum_t G[s, t] A_j[:, t, :]."""
    out = copy(mps)
    out[j] = np.einsum("st,atb->asb", G, mps[j])
    return out
