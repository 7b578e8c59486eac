"""Cost assembly, gradients and gradient descent -- oracle (test infrastructure only).

Paper:
  * global cost, Eq. (1): C_G = 1 - |<b|A|x>|^2 / <x|A^dagger A|x>;
  * local cost, Eq. (2) / expanded Eq. (4) with P_j = (I + Z_j)/2;
  * stage iii of Section II-C: with Psi = sum_lm c_l^* c_m beta_lm and
    E = sum_j sum_lm c_l^* c_m delta^j_lm (Z_j, not P_j),
    C_L = 1/2 - 1/2 Re[E / (n Psi)]  (Algorithm 1 Step 4c omits the Re; the
    text's form is used, E and Psi are real up to rounding anyway);
  * stage ii: the weights c_l^* c_l' of each term.

Gradients: the paper does not state its gradient method.  The oracle has two
routes: the exact parameter-shift rule applied to the expectation values Psi
and E (or G = |<b|A|x>|^2, itself an expectation value) followed by the
quotient rule, and central finite differences.  Gradient descent
theta <- theta - eta grad C is the optimizer of the parity trajectories.

Pins: Eq. (4) route == stage-iii route, terms route == dense route, cost = 0
at the exact solution, A = I special case, parameter shift == finite
differences, gradient descent against a quadratic whose iterates are known
in closed form (tests/test_oracle_cost.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import circuit as qc


def weights(coeffs: np.ndarray) -> np.ndarray:
    """w[l, m] = c_l^* c_m (Section II-C, stage ii)."""
    c = np.asarray(coeffs, dtype=np.complex128)
    return np.outer(np.conj(c), c)


def aggregate(coeffs, beta, other, kind: str):
    """(N, Psi) from the terms: N = E (local) or G (global)."""
    w = weights(coeffs)
    psi = np.sum(w * beta)
    if kind == "local":
        num = sum(np.sum(w * other[j]) for j in range(other.shape[0]))
    else:
        g = np.sum(np.asarray(coeffs) * other)
        num = abs(g) ** 2
    return num, psi


def cost_from_parts(num, psi, n: int, kind: str) -> float:
    """Stage iii closed form (local) or Eq. (1) (global)."""
    if kind == "local":
        return float(0.5 - 0.5 * (num / (n * psi)).real)
    return float(1.0 - (num / psi).real)


def cost_from_terms(coeffs, beta, other, n: int, kind: str) -> float:
    num, psi = aggregate(coeffs, beta, other, kind)
    return cost_from_parts(num, psi, n, kind)


def cost_local_eq4(coeffs, beta, delta) -> float:
    """Eq. (4) literally: numerators use P_j = (I + Z_j)/2, so the term for
    (l, m, j) is (beta_lm + delta^j_lm) / 2."""
    w = weights(coeffs)
    n = delta.shape[0]
    den = np.sum(w * beta)
    acc = 0.0
    for j in range(n):
        acc += (np.sum(w * (beta + delta[j]) / 2.0) / den).real
    return float(1.0 - acc / n)


# ------------------------------------------------------------ dense definitions

def ub_matrix(n: int, b_kind: str, b=None) -> np.ndarray:
    """Dense U_b: H^n for |+>^n, the Householder reflector for a real b."""
    if b_kind == "plus":
        H = qc.H2
        M = np.ones((1, 1), dtype=np.complex128)
        for _ in range(n):
            M = np.kron(M, H)
        return M
    return qc.householder_ub(b).astype(np.complex128)


def parts_dense(A_tilde, x, n: int, kind: str, b_kind="plus", b=None):
    """(N, Psi) straight from the definitions with dense matrices.

    Psi = <x|A^dagger A|x> = ||A x||^2.  Local: E = sum_j <A x|U_b Z_j U_b^dagger|A x>.
    Global: G = |<b|A|x>|^2.
    """
    y = A_tilde @ x
    psi = np.vdot(y, y)
    if kind == "local":
        U = ub_matrix(n, b_kind, b)
        u = U.conj().T @ y
        N = 1 << n
        e = 0.0
        for j in range(n):
            sign = 1.0 - 2.0 * ((np.arange(N) >> j) & 1)
            e += np.vdot(u, sign * u)
        return e, psi
    bb = qc.plus_vector(n) if b_kind == "plus" else np.asarray(b, dtype=np.complex128)
    g = np.vdot(bb, y)
    return abs(g) ** 2, psi


def cost_dense(A_tilde, x, n: int, kind: str, b_kind="plus", b=None) -> float:
    num, psi = parts_dense(A_tilde, x, n, kind, b_kind, b)
    return cost_from_parts(num, psi, n, kind)


def cost_local_eq2_dense(A_tilde, x, n: int, b_kind="plus", b=None) -> float:
    """Eq. (2) literally, with the projectors P_j = |0><0|_j."""
    y = A_tilde @ x
    psi = np.vdot(y, y).real
    U = ub_matrix(n, b_kind, b)
    u = U.conj().T @ y
    N = 1 << n
    acc = 0.0
    for j in range(n):
        proj = (((np.arange(N) >> j) & 1) == 0).astype(np.float64)
        acc += np.vdot(u, proj * u).real / psi
    return float(1.0 - acc / n)


# ------------------------------------------------------------ cost functions of theta

def parts_theta_dense(theta, A_tilde, n, layers, ent, kind, b_kind="plus", b=None):
    x = qc.ansatz_state(theta, n, layers, ent)
    return parts_dense(A_tilde, x, n, kind, b_kind, b)


def cost_theta_dense(theta, A_tilde, n, layers, ent, kind, b_kind="plus", b=None):
    num, psi = parts_theta_dense(theta, A_tilde, n, layers, ent, kind, b_kind, b)
    return cost_from_parts(num, psi, n, kind)


def grad_parameter_shift(parts_fn, theta, n: int, kind: str):
    """Exact gradient: shift rule on the expectation values, then quotient rule.

    For a gate RY(t) = exp(-i t Y / 2), d<O>/dt = (<O>(t + pi/2) - <O>(t - pi/2)) / 2.
    ``parts_fn(theta) -> (N, Psi)``.  Returns (C, grad).
    """
    theta = np.asarray(theta, dtype=np.float64)
    num0, psi0 = parts_fn(theta)
    num0, psi0 = num0.real if np.iscomplexobj(num0) else num0, psi0.real
    P = theta.shape[0]
    dnum = np.zeros(P)
    dpsi = np.zeros(P)
    for k in range(P):
        tp = theta.copy()
        tp[k] += math.pi / 2
        tm = theta.copy()
        tm[k] -= math.pi / 2
        np_, pp = parts_fn(tp)
        nm, pm = parts_fn(tm)
        dnum[k] = (np.real(np_) - np.real(nm)) / 2.0
        dpsi[k] = (np.real(pp) - np.real(pm)) / 2.0
    num0 = float(np.real(num0))
    psi0 = float(np.real(psi0))
    if kind == "local":
        C = 0.5 - 0.5 * num0 / (n * psi0)
        grad = -0.5 / n * (dnum * psi0 - num0 * dpsi) / psi0 ** 2
    else:
        C = 1.0 - num0 / psi0
        grad = -(dnum * psi0 - num0 * dpsi) / psi0 ** 2
    return C, grad


def grad_finite_difference(cost_fn, theta, h: float = 1e-4):
    """Central differences (C(t + h e_k) - C(t - h e_k)) / (2h)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(theta.shape[0]):
        tp = theta.copy()
        tp[k] += h
        tm = theta.copy()
        tm[k] -= h
        g[k] = (cost_fn(tp) - cost_fn(tm)) / (2.0 * h)
    return g


def parts_theta_circuits(theta, coeffs, xs, zs, n, layers, ent, kind, b_kind="plus", b=None):
    """(N, Psi) through every Hadamard-test circuit (the method's route)."""
    beta, other = qc.terms(theta, n, layers, ent, xs, zs, kind, b_kind, b)
    return aggregate(coeffs, beta, other, kind)


def gradient_descent(theta0, cost_grad_fn, eta: float, steps: int):
    """theta_{t+1} = theta_t - eta grad C(theta_t).  Returns (thetas, costs):
    thetas[t] is the iterate after t steps (thetas[0] = theta0) and costs[t]
    the cost at thetas[t]."""
    th = np.asarray(theta0, dtype=np.float64).copy()
    thetas = [th.copy()]
    costs = []
    for _ in range(steps):
        C, g = cost_grad_fn(th)
        costs.append(C)
        th = th - eta * g
        thetas.append(th.copy())
    costs.append(cost_grad_fn(th)[0])
    return np.array(thetas), np.array(costs)
