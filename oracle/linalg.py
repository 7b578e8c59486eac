"""Classical linear algebra around the solver -- oracle (test infrastructure only).

Paper:
  * Section III-A: the quantum solution is compared with the classical solution
    of direct inversion through the state fidelity F = |<psi|phi>|^2.
  * Section II-B, Eq. (6): for A_tilde = A + E and kappa ||E||/||A|| < 1,
    ||x - x_tilde|| / ||x|| <= kappa eps / (1 - kappa eps), eps = ||E||_2/||A||_2.
  * Section III-B: median over 64 normalised Gaussian right-hand sides of the
    relative solution error of the pruned system.

Solutions use LAPACK through numpy.linalg.solve.

Pins: the fidelity on hand-worked values (orthogonal pair, 1/2, (24/25)^2,
a pair orthogonal only under conjugation, global-phase invariance); the
perturbation bound and solution errors against the paper's Section III-B
figures (tests/test_oracle_cost.py, tests/test_oracle_pauli.py).
"""
from __future__ import annotations

import numpy as np


def solve(A, b):
    return np.linalg.solve(A, b)


def normalized(v):
    v = np.asarray(v, dtype=np.complex128)
    return v / np.linalg.norm(v)


def fidelity(u, v) -> float:
    """|<u|v>|^2 of the normalised vectors."""
    return float(abs(np.vdot(normalized(u), normalized(v))) ** 2)


def perturbation_bound(A, A_tilde) -> float:
    """Right-hand side of Eq. (6), or inf when kappa eps >= 1."""
    s = np.linalg.svd(A, compute_uv=False)
    kappa = s[0] / s[-1]
    eps = np.linalg.norm(A_tilde - A, 2) / s[0]
    ke = kappa * eps
    return float(ke / (1.0 - ke)) if ke < 1.0 else float("inf")


def relative_solution_errors(A, A_tilde, rhs):
    """e_j = ||A_tilde^{-1} b_j - A^{-1} b_j|| / ||A^{-1} b_j|| for each row b_j."""
    X = np.linalg.solve(A, rhs.T)
    Xt = np.linalg.solve(A_tilde, rhs.T)
    return np.linalg.norm(Xt - X, axis=0) / np.linalg.norm(X, axis=0)
