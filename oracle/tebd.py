"""TEBD with SVD truncation (oracle; test infrastructure only).

One slice of the time grid (Sec. II, Eq. 4):

    a_l = post_l . trunc[ Z_l . (pre_l a_{l-1}) ]

pre_l = post_l = R_l, the single-site half rotations, in the second-order
split; pre_l = I and post_l = X_l Y_l in the paper's first-order split
(oracle/gates.py).  Z_l is the two-site layer: ZZ phases in the ZZ crosstalk
model, the 4x4 bond exponentials G_b with Heisenberg crosstalk.  Z_l is
applied bond by bond in a sweep; after each bond the two-site tensor is split
by an SVD and compressed to at most chi singular values (the compression to a
maximum bond size after every step, Sec. II).  Every bond is split, also where
its gate is the identity, so the truncation is uniform.

Canonical form: an MPS entering a left-to-right sweep has its orthogonality
centre on site 0 and every other site right-isometric; the sweep leaves the
centre on site N-1 (sites 0..N-2 left-isometric), and a right-to-left sweep
mirrors this.  Slices alternate direction: forward slice l (1-based) sweeps
left to right when M - l is odd, backward slice l when M - l is even, so the
two sweeps of one slice always run in opposite directions and the last
forward slice ends with the centre on site 0, where the right-canonical
target starts the backward pass.  The Heisenberg bond gates of neighbouring
bonds do not commute, so their product is taken in the order of the forward
sweep (the bond visited first acts first) and the backward slice, sweeping
the other way, applies the exact adjoint of that product.  Two consecutive
forward slices visit the bonds in mirror order, a symmetric product, which
keeps the splitting of the bond terms at second order.

Truncation rule: singular values sorted in descending order, keep
    k = max(1, min(chi, #{i : sigma_i >= eps * sigma_1}))
and, with renormalisation on, replace sigma_{1..k} by sigma_{1..k} / ||sigma_{1..k}||_2.
"""
from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np

from . import gates
from .mps import MPS, copy


def keep_count(S: np.ndarray, chi: int, eps: float) -> int:
    if S.size == 0 or S[0] <= 0.0:
        return 1
    return max(1, min(int(chi), int(np.count_nonzero(S >= eps * S[0]))))


def _svd(m: np.ndarray):
    try:
        return np.linalg.svd(m, full_matrices=False)
    except np.linalg.LinAlgError:  # pragma: no cover - gesdd fallback
        import scipy.linalg
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


def split_two_site(theta: np.ndarray, chi: int, eps: float, renormalize: bool,
                   left_to_right: bool, stats: Optional[List[Dict]] = None):
    """Split theta (Dl, d, d, Dr) into (Dl, d, k) and (k, d, Dr) (d = 2 for
    qubit states, 4 for the operators of oracle/mpo.py).

    Left to right: left factor U (left-isometric), right factor diag(s) V^dagger
    (new centre).  Right to left: left factor U diag(s), right V^dagger.
    """
    Dl, d, _, Dr = theta.shape
    U, S, Vh = _svd(theta.reshape(Dl * d, d * Dr))
    k = keep_count(S, chi, eps)
    k = min(k, S.size)
    s = S[:k].copy()
    tot = float(np.sum(S ** 2))
    if stats is not None:
        # the cut is decided by chi (not by the cutoff) when more singular
        # values pass the cutoff than chi allows; only then can a near-tie
        # sigma_k ~ sigma_{k+1} make the truncated state non-unique.
        chi_cut = k < S.size and S[k] >= eps * S[0]
        stats.append(dict(k=k, discarded=float(np.sum(S[k:] ** 2)) / tot if tot > 0 else 0.0,
                          gap=float(S[k - 1] - S[k]) / S[0] if chi_cut else np.inf,
                          sigma=S.copy()))
    if renormalize:
        s = s / np.linalg.norm(s)
    if left_to_right:
        left = U[:, :k]
        right = s[:, None] * Vh[:k, :]
    else:
        left = U[:, :k] * s[None, :]
        right = Vh[:k, :]
    return left.reshape(Dl, d, k), right.reshape(k, d, Dr)


def bond_sweep(mps: MPS, gate, left_to_right: bool, chi: int, eps: float,
               renormalize: bool, stats: Optional[List[Dict]] = None,
               before=None, after=None) -> MPS:
    """Apply the two-site gates bond by bond in sweep order, each followed by
    a truncated split.  ``gate(b, theta)`` returns the gated theta
    (Dl, 2, 2, Dr).  ``before(b, state)`` / ``after(b, state)`` see the
    working MPS just before / just after bond b is updated."""
    out = copy(mps)
    N = len(out)
    order = range(N - 1) if left_to_right else range(N - 2, -1, -1)
    for b in order:
        if before is not None:
            before(b, out)
        theta = np.einsum("asb,btc->astc", out[b], out[b + 1])
        theta = gate(b, theta)
        out[b], out[b + 1] = split_two_site(theta, chi, eps, renormalize,
                                            left_to_right, stats)
        if after is not None:
            after(b, out)
    return out


def zz_layer(mps: MPS, phis: np.ndarray, left_to_right: bool, chi: int,
             eps: float, renormalize: bool,
             stats: Optional[List[Dict]] = None) -> MPS:
    """Apply prod_b exp(-i phis[b] Z_b Z_{b+1}) by a truncated bond sweep."""
    return bond_sweep(mps, lambda b, th: th * gates.zz_phase(phis[b])[None, :, :, None],
                      left_to_right, chi, eps, renormalize, stats)


def _apply4(G: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """theta'[a, s, t, c] = sum G[s, t, s', t'] theta[a, s', t', c]."""
    return np.einsum("stuv,auvc->astc", G, theta)


def forward_ltr(problem, l: int) -> bool:
    """Sweep direction of forward slice l (0-based): left to right when
    M - (l + 1) is odd."""
    return (problem.M - 1 - l) % 2 == 1


def _layer(problem, mps: MPS, l: int, k: int, ltr: bool, adjoint: bool, chi: int,
           stats, before=None, after=None) -> MPS:
    if gates.heisenberg(problem):
        G = gates.bond_gates(problem, k, l)
        if adjoint:   # (G_b)^dagger: swap (out, in) pairs and conjugate
            G = [np.conj(np.transpose(g, (2, 3, 0, 1))) for g in G]
        return bond_sweep(mps, lambda b, th: _apply4(G[b], th), ltr, chi, problem.eps,
                          problem.renormalize, stats, before, after)
    if before is not None or after is not None:
        raise ValueError("sweep hooks are only used with Heisenberg crosstalk")
    phis = problem.dt * gates.couplings(problem, k)[l]
    return zz_layer(mps, -phis if adjoint else phis, ltr, chi, problem.eps,
                    problem.renormalize, stats)


def rotation_layer(mps: MPS, G: np.ndarray) -> MPS:
    """A_j[:, s, :] <- sum_t G[j, s, t] A_j[:, t, :] on every site."""
    return [np.einsum("st,atb->asb", G[j], A) for j, A in enumerate(mps)]


def forward_slice(problem, mps: MPS, l: int, k: int, chi: Optional[int] = None,
                  stats=None, after=None) -> MPS:
    """a_l from a_{l-1}; ``l`` is 0-based (slice l+1 of the time grid).
    ``after(b, state)`` (Heisenberg crosstalk only) sees the two-site layer's
    working MPS after each bond update."""
    chi = problem.chi if chi is None else chi
    a = rotation_layer(mps, gates.slice_pre(problem, l))
    a = _layer(problem, a, l, k, forward_ltr(problem, l), False, chi, stats, after=after)
    return rotation_layer(a, gates.slice_post(problem, l))


def backward_slice(problem, mps: MPS, l: int, k: int, chi: Optional[int] = None,
                   stats=None, before=None) -> MPS:
    """b_l = U_l^dagger b_{l+1} (with truncation); ``l`` is 0-based.
    ``before(b, state)`` (Heisenberg crosstalk only) sees the working MPS
    before each bond update."""
    chi = problem.chi if chi is None else chi
    dag = lambda G: np.conj(np.transpose(G, (0, 2, 1)))
    b = rotation_layer(mps, dag(gates.slice_post(problem, l)))
    b = _layer(problem, b, l, k, not forward_ltr(problem, l), True, chi, stats, before=before)
    return rotation_layer(b, dag(gates.slice_pre(problem, l)))


def evolve(problem, mps: MPS, k: int, l_begin: int = 0,
           l_end: Optional[int] = None, adjoint: bool = False,
           chi: Optional[int] = None, keep_all: bool = False, stats=None):
    """Apply slices l_begin..l_end-1 (0-based) forward, or, with ``adjoint``,
    the adjoint slices l_end-1 down to l_begin.  Returns the final MPS, or the
    list of all intermediate states when ``keep_all``."""
    l_end = problem.M if l_end is None else l_end
    states = [mps]
    cur = mps
    if not adjoint:
        for l in range(l_begin, l_end):
            cur = forward_slice(problem, cur, l, k, chi, stats)
            if keep_all:
                states.append(cur)
    else:
        for l in range(l_end - 1, l_begin - 1, -1):
            cur = backward_slice(problem, cur, l, k, chi, stats)
            if keep_all:
                states.append(cur)
    return states if keep_all else cur
