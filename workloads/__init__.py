"""Seeded synthetic workloads for ensemble-robust GRAPE on qubit-chain MPS.

This module only draws random numbers and lays out arrays: piecewise-constant
control amplitudes, crosstalk samples, product-state inputs and the target MPS
tensors of the tasks in Secs. III-IV of the paper (parallel X, parallel CNOT,
GHZ).  It holds none of the propagation, truncation, overlap or gradient
arithmetic.  Both the CPU oracle and the HIP library consume what it returns,
and neither side's code lives here.

Conventions shared by every consumer
------------------------------------
* Sites j = 0..N-1 of an open chain, bond b couples (b, b+1).
* Computational basis |0> <-> Z = +1.
* A site tensor is a complex128 array of shape (D_l, 2, D_r).
* Controls are float64: ``ux[l, j]``, ``uy[l, j]`` (shape (M, N)) and
  ``uzz[l, b]`` (shape (M, N-1)); slice l = 0..M-1 here is slice l+1 of the
  paper's 1-based time grid (Sec. II, Eq. 4).
* ``zz_mask[b]`` marks bonds that carry the controllable coupling u^zz,
  ``xt_mask[b]`` marks bonds that carry the static crosstalk (Sec. III,
  Eqs. 8-9).
* Crosstalk model ``xt_model``: ``"zz"`` keeps the J_j Z_j Z_{j+1} part of
  Eq. 9 and ``J[k, b]`` is its strength for noise sample k on bond b;
  ``"heisenberg"`` is the full Eq. 9, J^x XX + J^y YY + J^z ZZ on every bond,
  and ``J[k, b, :]`` holds (J^x, J^y, J^z).  Static in time; trajectory t of
  a batch is (k, r) = (t // R, t % R).
* Targets are returned right-canonical (every site right-isometric, the first
  site carrying the norm, which is 1).
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np

__all__ = ["Problem", "CONFIGS", "make_problem", "haar_qubits", "heisenberg_ground_state",
           "heisenberg_mps", "serving_mix"]


@dataclasses.dataclass
class Problem:
    """A complete fidelity+gradient request: model, controls, ensemble, data."""

    N: int
    M: int
    T: float
    chi: int
    eps: float
    renormalize: bool
    ux: np.ndarray          # (M, N) float64
    uy: np.ndarray          # (M, N) float64
    uzz: np.ndarray         # (M, N-1) float64
    zz_mask: np.ndarray     # (N-1,) uint8
    xt_mask: np.ndarray     # (N-1,) uint8
    J: np.ndarray           # (K, N-1) or, Heisenberg, (K, N-1, 3) float64; 0 off xt_mask
    inputs: np.ndarray      # (R, N, 2) complex128 product-state qubits
    targets: List[List[np.ndarray]]  # R target MPS, each N tensors (Dl,2,Dr)
    task: str = "x"
    name: str = ""
    order: int = 2          # Trotter split: 2 (R Z R) or 1 (the paper's X Y Z)
    xt_model: str = "zz"    # crosstalk: "zz" or "heisenberg" (XX + YY + ZZ)

    @property
    def dt(self) -> float:
        return self.T / self.M

    @property
    def K(self) -> int:
        return int(self.J.shape[0])

    @property
    def R(self) -> int:
        return int(self.inputs.shape[0])

    @property
    def n_traj(self) -> int:
        return self.K * self.R

    def subset(self, ks=None, rs=None) -> "Problem":
        """Same controls, a sub-ensemble: noise samples ``ks``, inputs ``rs``."""
        ks = list(range(self.K)) if ks is None else list(ks)
        rs = list(range(self.R)) if rs is None else list(rs)
        return dataclasses.replace(
            self,
            J=self.J[ks].copy(),
            inputs=self.inputs[rs].copy(),
            targets=[[a.copy() for a in self.targets[r]] for r in rs],
        )


# Workload shapes.  T for the gate tasks is 10 (units of 1/max drive); GHZ uses
# T = N * tau_g / 8 with tau_g = 2 pi (coupling scale 1), the duration rule of
# Sec. IV.
CONFIGS = {
    "xgate_n8": dict(task="x", N=8, M=50, T=10.0, chi=16, K=16, R=4,
                     sigma=0.02, seed=0),
    "xgate_n50": dict(task="x", N=50, M=100, T=10.0, chi=32, K=64, R=4,
                      sigma=0.02, seed=1),
    "cnot_n50": dict(task="cnot", N=50, M=200, T=10.0, chi=64, K=128, R=8,
                     sigma=0.02, seed=2),
    "ghz_n30": dict(task="ghz", N=30, M=300, T=30 * 2 * math.pi / 8, chi=128,
                    K=256, R=1, sigma=0.05, seed=3),
}


def haar_qubits(rng: np.random.Generator, shape) -> np.ndarray:
    """Independent Haar-random single-qubit states, normalised, shape (..., 2)."""
    g = rng.standard_normal(tuple(shape) + (2, 2))
    v = g[..., 0] + 1j * g[..., 1]
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _masks(task: str, N: int):
    b = np.arange(N - 1)
    if task in ("x", "identity"):
        return np.zeros(N - 1, np.uint8), np.ones(N - 1, np.uint8)
    if task == "cnot":
        # u^zz on the pair bonds (2p, 2p+1), crosstalk on the bonds between
        # pairs (Sec. III, Eq. 11 with 0-based sites).
        return (b % 2 == 0).astype(np.uint8), (b % 2 == 1).astype(np.uint8)
    if task in ("ghz", "heisenberg", "state"):
        return np.ones(N - 1, np.uint8), np.ones(N - 1, np.uint8)
    raise ValueError(f"unknown task {task!r}")


def _product_mps(vecs: np.ndarray) -> List[np.ndarray]:
    return [np.asarray(v, np.complex128).reshape(1, 2, 1).copy() for v in vecs]


def _cnot_pair_mps(v0: np.ndarray, v1: np.ndarray) -> List[np.ndarray]:
    """Right-canonical bond-2 MPS of CNOT(control 0, target 1) |v0>|v1>."""
    psi = np.zeros((2, 2), np.complex128)
    for s0 in range(2):
        for s1 in range(2):
            psi[s0, s1 ^ s0] = v0[s0] * v1[s1]
    # psi = L @ Q with Q unitary: QR of psi^T gives psi = R^T Q^T.
    q, r = np.linalg.qr(psi.T)
    left = r.T            # (s0, beta)
    right = q.T           # (beta, s1), orthonormal rows
    return [left.reshape(1, 2, 2).copy(), right.reshape(2, 2, 1).copy()]


def ghz_mps(N: int) -> List[np.ndarray]:
    """The bond-2 GHZ MPS written out in Sec. IV (Eqs. 14-15).

    The first site is a row vector, the last a column vector and the middle
    sites are the projectors diag(1,0), diag(0,1); this form is already
    right-canonical with unit norm.
    """
    h = 2.0 ** -0.5
    first = np.zeros((1, 2, 2), np.complex128)
    first[0, 0, 0] = h
    first[0, 1, 1] = h
    mid = np.zeros((2, 2, 2), np.complex128)
    mid[0, 0, 0] = 1.0
    mid[1, 1, 1] = 1.0
    last = np.zeros((2, 2, 1), np.complex128)
    last[0, 0, 0] = 1.0
    last[1, 1, 0] = 1.0
    return [first] + [mid.copy() for _ in range(N - 2)] + [last]


@functools.lru_cache(maxsize=4)
def heisenberg_ground_state(N: int, tol: float = 1e-12):
    """Ground state of the open chain H = sum_j (XX + YY + ZZ)_{j,j+1} on N
    qubits (even N), by Lanczos (ARPACK) in the S^z = 0 sector, returned as a
    dense real vector of length 2^N (bit j of the index is qubit j, 0 = |0>),
    with its energy.  Used as a state-preparation target (Sec. IV)."""
    import scipy.sparse.linalg as sla
    if N % 2:
        raise ValueError("even N required")
    idx = np.arange(1 << N, dtype=np.int64)
    pop = np.zeros(1 << N, np.int64)
    for j in range(N):
        pop += (idx >> j) & 1
    basis = idx[pop == N // 2]
    n = basis.size
    diag = np.zeros(n)
    hops = []
    for b in range(N - 1):
        differ = ((basis >> b) ^ (basis >> (b + 1))) & 1
        diag += 1.0 - 2.0 * differ
        src = np.nonzero(differ)[0]
        dst = np.searchsorted(basis, basis[src] ^ (3 << b))
        hops.append((src, dst))

    def matvec(x):
        x = np.asarray(x).reshape(-1)
        y = diag * x
        for src, dst in hops:
            y[dst] += 2.0 * x[src]      # XX + YY swaps an antiparallel pair
        return y

    op = sla.LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    v0 = np.random.default_rng(N).standard_normal(n)
    w, v = sla.eigsh(op, k=1, which="SA", v0=v0, tol=tol)
    full = np.zeros(1 << N)
    full[basis] = v[:, 0]
    full /= np.linalg.norm(full)
    return full, float(w[0])


def heisenberg_mps(N: int = 20, chi: int = 64, eps: float = 1e-12) -> List[np.ndarray]:
    """The Heisenberg ground state compressed to an MPS of bond dimension at
    most chi by successive SVDs from the right (keeping the singular values
    >= eps sigma_1), right-canonical with unit norm."""
    psi, _ = heisenberg_ground_state(N)
    # site order: site 0 is the most significant index of the reshaped
    # vector, so bit j of the index must be qubit N-1-j: reverse the bits
    t = psi.reshape((2,) * N).transpose(tuple(range(N - 1, -1, -1))).reshape(-1)
    rest = t.astype(np.complex128)
    sites: List[np.ndarray] = []
    dr = 1
    for j in range(N - 1, 0, -1):
        mat = rest.reshape(-1, 2 * dr)
        U, S, Vh = np.linalg.svd(mat, full_matrices=False)
        k = int(max(1, min(chi, np.sum(S >= eps * S[0]))))
        sites.append(Vh[:k].reshape(k, 2, dr).copy())
        rest = U[:, :k] * S[:k]
        dr = k
    first = rest.reshape(1, 2, dr)
    sites.append(first / np.linalg.norm(first))
    return sites[::-1]


def _targets(task: str, inputs: np.ndarray, N: int) -> List[List[np.ndarray]]:
    out = []
    for vecs in inputs:
        if task == "x":
            out.append(_product_mps(vecs[:, ::-1]))
        elif task == "identity":
            out.append(_product_mps(vecs))
        elif task == "cnot":
            mps: List[np.ndarray] = []
            for p in range(N // 2):
                mps += _cnot_pair_mps(vecs[2 * p], vecs[2 * p + 1])
            if N % 2:
                mps += _product_mps(vecs[-1:])
            out.append(mps)
        elif task == "ghz":
            out.append(ghz_mps(N))
        elif task == "heisenberg":
            out.append([A.copy() for A in heisenberg_mps(N, 64)])
        else:
            raise ValueError(task)
    return out


def make_problem(name: Optional[str] = None, *, task: Optional[str] = None,
                 N: Optional[int] = None, M: Optional[int] = None,
                 T: Optional[float] = None, chi: Optional[int] = None,
                 K: Optional[int] = None, R: Optional[int] = None,
                 sigma: Optional[float] = None, seed: Optional[int] = None,
                 eps: float = 1e-12, renormalize: bool = True,
                 controls: str = "uniform", amp: float = 1.0,
                 crosstalk: float = 1.0, order: int = 2, xt_model: str = "zz",
                 delta_j: float = 0.05) -> Problem:
    """Build a seeded synthetic problem.

    ``name`` selects one of ``CONFIGS`` (keyword arguments override it).
    ``controls``: ``"uniform"`` draws every amplitude from U(-amp, amp);
    ``"pi_pulse"`` puts the global pi pulse u^x = pi/T on every site and adds
    U(-amp, amp) to all amplitudes (a near-optimal X-gate pulse, so that F is
    O(1) even at N = 50); ``"zero"`` sets every control to 0.
    ``crosstalk`` scales the drawn J (0 disables the noise).  ``order`` picks
    the Trotter split of a slice (2: second order; 1: the paper's first-order
    X Y Z product).  ``xt_model="heisenberg"`` draws the paper's noise model
    instead of the ZZ one: J^x, J^y, J^z independent and uniform in
    [-delta_j, delta_j] on every bond (Sec. II; Sec. III, Eq. 9); ``sigma`` is
    then unused.
    The seed is split with ``SeedSequence(seed).spawn(3)`` into the streams for
    controls, crosstalk and inputs.
    """
    cfg = dict(CONFIGS[name]) if name is not None else dict(
        task="x", N=8, M=50, T=10.0, chi=16, K=16, R=4, sigma=0.02, seed=0)
    for key, val in dict(task=task, N=N, M=M, T=T, chi=chi, K=K, R=R,
                         sigma=sigma, seed=seed).items():
        if val is not None:
            cfg[key] = val
    task, N, M, T, chi, K, R, sigma, seed = (
        cfg["task"], int(cfg["N"]), int(cfg["M"]), float(cfg["T"]),
        int(cfg["chi"]), int(cfg["K"]), int(cfg["R"]), float(cfg["sigma"]),
        int(cfg["seed"]))
    if N < 2:
        raise ValueError("N >= 2 required")
    ss = np.random.SeedSequence(seed).spawn(3)
    rc, rj, ri = (np.random.default_rng(s) for s in ss)
    zz_mask, xt_mask = _masks(task, N)
    if xt_model not in ("zz", "heisenberg"):
        raise ValueError(f"unknown crosstalk model {xt_model!r}")
    if xt_model == "heisenberg":
        xt_mask = np.ones(N - 1, np.uint8)   # Eq. 9 sums over every bond

    if controls == "uniform":
        ux = rc.uniform(-amp, amp, (M, N))
        uy = rc.uniform(-amp, amp, (M, N))
        uzz = rc.uniform(-amp, amp, (M, N - 1))
    elif controls == "pi_pulse":
        ux = math.pi / T + rc.uniform(-amp, amp, (M, N))
        uy = rc.uniform(-amp, amp, (M, N))
        uzz = rc.uniform(-amp, amp, (M, N - 1))
    elif controls == "zero":
        ux = np.zeros((M, N))
        uy = np.zeros((M, N))
        uzz = np.zeros((M, N - 1))
    else:
        raise ValueError(controls)
    uzz = uzz * zz_mask[None, :]

    if xt_model == "heisenberg":
        J = rj.uniform(-delta_j, delta_j, (K, N - 1, 3)) * crosstalk * xt_mask[None, :, None]
    else:
        J = rj.normal(0.0, sigma, (K, N - 1)) * crosstalk * xt_mask[None, :]

    if task in ("ghz", "heisenberg"):
        inputs = np.zeros((R, N, 2), np.complex128)
        inputs[..., 0] = 1.0
    else:
        inputs = haar_qubits(ri, (R, N))
    targets = _targets(task, inputs, N)
    return Problem(N=N, M=M, T=float(T), chi=int(chi), eps=float(eps),
                   renormalize=bool(renormalize), ux=ux, uy=uy, uzz=uzz,
                   zz_mask=zz_mask, xt_mask=xt_mask, J=J, inputs=inputs,
                   targets=targets, task=task, name=name or task, order=int(order),
                   xt_model=xt_model)


# Request mix of the serving workload: N in {10, 20, 30, 50}, chi in
# {16, 32, 64, 128}, K in {8, 32, 128}, M uniform in 100..300, task in
# {X gate, CNOT, GHZ, Heisenberg ground state (N = 20)}; R = 4 inputs for
# gates, 1 for states; T = 10 for gates, N 2 pi / 8 for GHZ, N 2 pi / 2 for
# the Heisenberg state (Sec. IV time scales); crosstalk sigma 0.02 for gates,
# 0.05 for states.
def serving_mix(n: int, seed: int = 4, ks=(8, 32, 128), ns=(10, 20, 30, 50),
                chis=(16, 32, 64, 128), m_range=(100, 300)) -> List[dict]:
    """n request specs (keyword arguments of make_problem) drawn from the mix."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        task = ("x", "cnot", "ghz", "heisenberg")[int(rng.integers(4))]
        N = 20 if task == "heisenberg" else int(rng.choice(ns))
        gate = task in ("x", "cnot")
        T = 10.0 if gate else (N * 2 * math.pi / 8 if task == "ghz" else N * 2 * math.pi / 2)
        out.append(dict(task=task, N=N, chi=int(rng.choice(chis)), K=int(rng.choice(ks)),
                        M=int(rng.integers(m_range[0], m_range[1] + 1)), R=4 if gate else 1,
                        T=T, sigma=0.02 if gate else 0.05, seed=1000 * seed + i))
    return out
