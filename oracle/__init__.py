"""CPU oracle for the ensemble-robust GRAPE hot path on qubit-chain MPS.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything in
this package.  The HIP library and its Python binding never do, and this
package imports nothing from them.

What it computes, in the paper's order (Le, Mintert, Ginossar, "Mitigating
many-body quantum crosstalk with tensor-network robust control"):

* ``gates``       single-site half-slice rotations and their control
                  derivatives, ZZ phases and Heisenberg bond gates (Sec. II,
                  Eq. 4; Sec. III, Eqs. 8-9).
* ``mps``         product states, overlaps by transfer matrices, right
                  canonicalisation by QR (Sec. II; Sec. IV initial state).
* ``tebd``        the truncated two-site SVD update and the second-order
                  (Strang) slice, forward and adjoint (Sec. II, Eq. 4 and the
                  SVD compression to a maximum bond size).
* ``grape``       ensemble fidelity (Sec. II, Eq. 7) and its exact adjoint
                  gradient (App. A, Eqs. A1-A2).
* ``mpo``         the gate objective |tr(U_T^dag U)/2^n|^2 with the
                  propagator as an MPO, and its adjoint gradient (Sec. II,
                  Eqs. 5-6; App. A).
* ``statevector`` dense references used to pin the above at N <= 12.

Everything is complex128 / float64.  Plain, slow and written to be read next
to the paper: no blocking, fusion or reordering beyond what the definitions
state.  Pins live in ``tests/test_oracle_*.py``.

Readings taken where the paper is silent (each is listed with its reason in
the design notes of the repository): Strang splitting R Z R per slice with the
drive combined per site; relative singular-value cutoff sigma_i >= eps *
sigma_1 capped at chi, k >= 1; renormalisation after each truncation; sweep
direction alternating by slice, forward and backward opposite; Heisenberg
bond gates in sweep order with mid-sweep u^zz insertions; the final forward
overlap multiplies every dO in dF.
"""

from . import gates, mps, tebd, grape, mpo, statevector  # noqa: F401

__all__ = ["gates", "mps", "tebd", "grape", "mpo", "statevector"]
