"""Dense state-vector references (oracle; test infrastructure only, N <= ~12).

* ``strang_states``: the same second-order circuit R Z R per slice as the MPS
  code, applied to a 2^N vector, no truncation (with Heisenberg crosstalk, Z
  is the product of the 4x4 bond gates in the slice's sweep order).
* ``exact_states``: piecewise-constant exact propagation
  psi_l = expm(-i H_l dt) psi_{l-1} with H_l = sum_j (ux X + uy Y)_j / 2 +
  sum_b c_b Z_b Z_{b+1} (Sec. II, Eq. 1 with Sec. III, Eq. 8; plus
  J^x XX + J^y YY on each bond with Heisenberg crosstalk, Eq. 9), for the
  second-order error check.
* ``adjoint_gradient``: dO/du of the dense Strang circuit from dense forward
  and backward vectors and the same insertion operators as the MPS adjoint.

Site 0 is the most significant qubit of the vector index.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import gates


def kron_vec(vecs) -> np.ndarray:
    v = np.ones(1, np.complex128)
    for q in vecs:
        v = np.kron(v, np.asarray(q, np.complex128))
    return v


def apply_local(psi: np.ndarray, N: int, j: int, G: np.ndarray) -> np.ndarray:
    t = psi.reshape((2 ** j, 2, 2 ** (N - j - 1)))
    return np.einsum("st,atb->asb", G, t).reshape(-1)


def apply_two(psi: np.ndarray, N: int, b: int, G: np.ndarray) -> np.ndarray:
    """Apply the (2, 2, 2, 2) gate G[s, t, s', t'] to sites (b, b+1)."""
    t = psi.reshape((2 ** b, 2, 2, 2 ** (N - b - 2)))
    return np.einsum("stuv,auvc->astc", G, t).reshape(-1)


def bond_layer(psi: np.ndarray, problem, k: int, l: int) -> np.ndarray:
    """Heisenberg two-site layer of forward slice l: the bond gates in the
    slice's sweep order, the first visited bond acting first."""
    N = problem.N
    G = gates.bond_gates(problem, k, l)
    ltr = (problem.M - 1 - l) % 2 == 1
    for b in (range(N - 1) if ltr else range(N - 2, -1, -1)):
        psi = apply_two(psi, N, b, G[b])
    return psi


def apply_all_sites(psi: np.ndarray, N: int, Gs) -> np.ndarray:
    for j in range(N):
        psi = apply_local(psi, N, j, Gs[j])
    return psi


def zvalues(N: int) -> np.ndarray:
    """z[idx, j] = +1 / -1 for bit j (site j) of basis index idx."""
    idx = np.arange(2 ** N)
    bits = (idx[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1
    return 1.0 - 2.0 * bits


def zz_diagonal(phis: np.ndarray, N: int) -> np.ndarray:
    z = zvalues(N)
    e = np.zeros(2 ** N)
    for b in range(N - 1):
        e += phis[b] * z[:, b] * z[:, b + 1]
    return np.exp(-1j * e)


def strang_states(problem, k: int, psi0: np.ndarray):
    """States after every slice of the dense circuit U_l = post Z pre (the
    split of ``problem.order``, second order by default)."""
    N, M, dt = problem.N, problem.M, problem.dt
    c = gates.couplings(problem, k)
    out = [psi0.copy()]
    psi = psi0.copy()
    for l in range(M):
        psi = apply_all_sites(psi, N, gates.slice_pre(problem, l))
        if gates.heisenberg(problem):
            psi = bond_layer(psi, problem, k, l)
        else:
            psi = zz_diagonal(dt * c[l], N) * psi
        psi = apply_all_sites(psi, N, gates.slice_post(problem, l))
        out.append(psi)
    return out


def hamiltonian(problem, k: int, l: int) -> scipy.sparse.csr_matrix:
    N = problem.N
    dim = 2 ** N
    c = gates.couplings(problem, k)[l]
    z = zvalues(N)
    diag = np.zeros(dim)
    for b in range(N - 1):
        diag += c[b] * z[:, b] * z[:, b + 1]
    H = scipy.sparse.diags(diag.astype(np.complex128)).tocsr()
    if gates.heisenberg(problem):
        J = problem.J[k]
        for b in range(N - 1):
            op = problem.xt_mask[b] * (J[b, 0] * gates.XX + J[b, 1] * gates.YY)
            H = H + scipy.sparse.kron(scipy.sparse.identity(2 ** b),
                                      scipy.sparse.kron(op, scipy.sparse.identity(2 ** (N - b - 2))))
    for j in range(N):
        loc = 0.5 * (problem.ux[l, j] * gates.X + problem.uy[l, j] * gates.Y)
        op = scipy.sparse.kron(scipy.sparse.identity(2 ** j),
                               scipy.sparse.kron(loc, scipy.sparse.identity(2 ** (N - j - 1))))
        H = H + op
    return H.tocsr()


def exact_final(problem, k: int, psi0: np.ndarray) -> np.ndarray:
    psi = psi0.copy()
    for l in range(problem.M):
        H = hamiltonian(problem, k, l)
        psi = scipy.sparse.linalg.expm_multiply(-1j * problem.dt * H, psi)
    return psi


def adjoint_gradient(problem, k: int, psi0: np.ndarray, target: np.ndarray):
    """(O, dux, duy, duzz) of the dense circuit (second or first order, ZZ
    crosstalk)."""
    if gates.heisenberg(problem):
        raise NotImplementedError("dense adjoint of the ZZ crosstalk model only")
    N, M, dt = problem.N, problem.M, problem.dt
    c = gates.couplings(problem, k)
    a = strang_states(problem, k, psi0)
    O = np.vdot(target, a[M])
    dux = np.zeros((M, N), np.complex128)
    duy = np.zeros((M, N), np.complex128)
    duzz = np.zeros((M, N - 1), np.complex128)
    z = zvalues(N)
    dag = lambda G: np.conj(np.transpose(G, (0, 2, 1)))
    b = target.copy()                                   # b_{M+1}
    for l in range(M, -1, -1):
        al = a[l]
        if l >= 1:
            s = l - 1
            for j in range(N):
                _, P, _, (dx, dy) = gates.site_factors(problem, s, j)
                dux[s, j] += np.vdot(b, apply_local(al, N, j, dx @ P.conj().T))
                duy[s, j] += np.vdot(b, apply_local(al, N, j, dy @ P.conj().T))
            post = gates.slice_post(problem, s)
            for bd in range(N - 1):
                if not problem.zz_mask[bd]:
                    continue
                # post (Z Z) post^dagger on the bond
                v = apply_local(al, N, bd, post[bd].conj().T)
                v = apply_local(v, N, bd + 1, post[bd + 1].conj().T)
                v = z[:, bd] * z[:, bd + 1] * v
                v = apply_local(v, N, bd, post[bd])
                v = apply_local(v, N, bd + 1, post[bd + 1])
                duzz[s, bd] += -1j * dt * np.vdot(b, v)
        if l <= M - 1 and gates.order(problem) == 2:
            s = l
            for j in range(N):
                Q, _, (dx, dy), _ = gates.site_factors(problem, s, j)
                dux[s, j] += np.vdot(b, apply_local(al, N, j, Q.conj().T @ dx))
                duy[s, j] += np.vdot(b, apply_local(al, N, j, Q.conj().T @ dy))
        if l >= 1:
            s = l - 1
            b = apply_all_sites(b, N, dag(gates.slice_post(problem, s)))
            b = np.conj(zz_diagonal(dt * c[s], N)) * b
            b = apply_all_sites(b, N, dag(gates.slice_pre(problem, s)))
    return O, dux, duy, duzz
