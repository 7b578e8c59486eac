"""Pins of the oracle's cost assembly and gradients (CPU only)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import circuit as qc
from oracle import cost as oc
from oracle import linalg as ola
from oracle import pauli as op
from workloads import plus_state, random_unit_vector, theta_uniform, toeplitz


def _system(n=3, a=1.0, b=-0.4, tau=0.01):
    A = toeplitz(n, a, b)
    C = op.decompose_fwht(A)
    keep = op.select_tau(C, tau)
    c, xs, zs = op.kept_terms(C, keep)
    At = op.reconstruct(c, xs, zs, n)
    return A, At, c, xs, zs


@pytest.mark.parametrize("b_kind", ["plus", "vector"])
def test_terms_route_equals_dense_definitions(b_kind):
    """Cost from the Hadamard-test terms (stage ii/iii) == cost from the dense
    definitions (Eq. (1) / Eq. (2)), both cost kinds."""
    n, layers = 3, 2
    A, At, c, xs, zs = _system(n)
    b = random_unit_vector(1 << n, seed=3) if b_kind == "vector" else None
    th = theta_uniform(n * layers, seed=0)
    x = qc.ansatz_state(th, n, layers)
    for kind in ("global", "local"):
        beta, other = qc.terms(th, n, layers, "cz", xs, zs, kind, b_kind, b)
        c_terms = oc.cost_from_terms(c, beta, other, n, kind)
        c_dense = oc.cost_dense(At, x, n, kind, b_kind, b)
        assert abs(c_terms - c_dense) < 1e-13
        if kind == "local":
            assert abs(oc.cost_local_eq4(c, beta, other) - c_terms) < 1e-14
            assert abs(oc.cost_local_eq2_dense(At, x, n, b_kind, b) - c_dense) < 1e-14


@pytest.mark.parametrize("kind", ["global", "local"])
@pytest.mark.parametrize("b_kind", ["plus", "vector"])
def test_cost_vanishes_at_exact_solution(kind, b_kind):
    n = 3
    A, At, c, xs, zs = _system(n)
    b = plus_state(n) if b_kind == "plus" else random_unit_vector(1 << n, seed=4)
    xt = np.linalg.solve(At, b.astype(complex))
    xt /= np.linalg.norm(xt)
    val = oc.cost_dense(At, xt, n, kind, b_kind, None if b_kind == "plus" else b)
    assert abs(val) < 1e-14


def test_identity_matrix_global_cost_is_infidelity():
    """A = I (one term): C_G = 1 - |<b|x>|^2."""
    n, layers = 3, 2
    th = theta_uniform(n * layers, seed=5)
    x = qc.ansatz_state(th, n, layers)
    b = random_unit_vector(1 << n, seed=6)
    beta, gamma = qc.terms(th, n, layers, "cz", [0], [0], "global", "vector", b)
    val = oc.cost_from_terms(np.array([1.0 + 0j]), beta, gamma, n, "global")
    assert abs(val - (1.0 - abs(np.vdot(b, x)) ** 2)) < 1e-14


@pytest.mark.parametrize("kind", ["global", "local"])
def test_parameter_shift_equals_finite_difference(kind):
    n, layers = 3, 2
    A, At, c, xs, zs = _system(n)
    th = theta_uniform(n * layers, seed=2)
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", kind)
    C0, g_ps = oc.grad_parameter_shift(parts, th, n, kind)
    g_fd = oc.grad_finite_difference(lambda t: oc.cost_theta_dense(t, At, n, layers, "cz", kind), th, 1e-4)
    assert abs(C0 - oc.cost_theta_dense(th, At, n, layers, "cz", kind)) < 1e-15
    assert np.max(np.abs(g_ps - g_fd)) < 1e-7


def test_parameter_shift_through_circuits_equals_dense_route():
    """The shift rule evaluated through every Hadamard-test circuit agrees with
    the dense route (n = 3, global cost, the small workload's system)."""
    n, layers = 3, 2
    A, At, c, xs, zs = _system(n)
    th = theta_uniform(n * layers, seed=0)
    p_circ = lambda t: oc.parts_theta_circuits(t, c, xs, zs, n, layers, "cz", "global")
    p_dense = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "global")
    C1, g1 = oc.grad_parameter_shift(p_circ, th, n, "global")
    C2, g2 = oc.grad_parameter_shift(p_dense, th, n, "global")
    assert abs(C1 - C2) < 1e-13 and np.max(np.abs(g1 - g2)) < 1e-13


def test_gradient_descent_decreases_cost():
    n, layers = 3, 2
    A, At, c, xs, zs = _system(n)
    th0 = theta_uniform(n * layers, seed=0)
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "global")
    thetas, costs = oc.gradient_descent(th0, lambda t: oc.grad_parameter_shift(parts, t, n, "global"), 0.1, 50)
    assert thetas.shape == (51, 6) and costs.shape == (51,)
    assert costs[-1] < costs[0]


def test_convergence_reaches_fidelity_cnot_ladder():
    """With no pruning (L = 2^n at n = 3) and the CNOT ladder, minimising the
    cost reaches fidelity >= 0.9999 against the classical solution (Section
    III-A reports > 0.9999 at four qubits)."""
    n, layers = 3, 2
    A = toeplitz(n, 1.0, -0.4)
    C = op.decompose_fwht(A)
    keep = op.select_tau(C, 0.0)
    c, xs, zs = op.kept_terms(C, keep)
    assert len(keep) == 1 << n
    At = op.reconstruct(c, xs, zs, n)
    b = plus_state(n)
    xsol = ola.solve(A, b)
    best = 0.0
    for seed in range(4):
        th0 = theta_uniform(n * layers, seed=seed)
        f = lambda t: oc.cost_theta_dense(t, At, n, layers, "cnot", "global")
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cnot", "global")
        g = lambda t: oc.grad_parameter_shift(parts, t, n, "global")[1]
        res = minimize(f, th0, jac=g, method="L-BFGS-B", options=dict(maxiter=500, gtol=1e-12, ftol=1e-15))
        x = qc.ansatz_state(res.x, n, layers, "cnot")
        best = max(best, ola.fidelity(x, xsol))
    assert best >= 0.9999


def test_cz_ladder_cannot_reach_fidelity_small_case():
    """The RY + CZ-ladder ansatz is real and its reachable set at n = 3 misses
    the Toeplitz solution: the best fidelity over several restarts stays
    below 0.995 (a property of the ansatz, reported, not a defect)."""
    n, layers = 3, 2
    A = toeplitz(n, 1.0, -0.4)
    b = plus_state(n)
    xsol = ola.solve(A, b)
    best = 0.0
    for seed in range(4):
        th0 = theta_uniform(n * layers, seed=seed)
        f = lambda t: -ola.fidelity(qc.ansatz_state(t, n, layers, "cz"), xsol)
        res = minimize(f, th0, method="BFGS", options=dict(maxiter=400))
        best = max(best, -res.fun)
    assert best < 0.995


def test_fidelity_hand_values():
    """F = |<u|v>|^2 of the normalised vectors (Section III-A), on cases worked
    by hand: orthogonal states, a 45-degree pair (1/2), the pair (3,4)/(4,3)
    whose normalised overlap is 24/25, a pair that is orthogonal only because
    the first vector is conjugated, and invariance under a global phase."""
    assert ola.fidelity([1.0, 0.0], [0.0, 1.0]) == 0.0
    assert abs(ola.fidelity([1.0, 0.0], [1.0, 1.0]) - 0.5) < 1e-15
    assert abs(ola.fidelity([3.0, 4.0], [4.0, 3.0]) - 576.0 / 625.0) < 1e-15
    assert abs(ola.fidelity([1.0, 1j], [1.0, -1j])) < 1e-15
    assert abs(ola.fidelity([1.0, 1j], [1.0, 1j]) - 1.0) < 1e-15
    u = np.array([0.3, -1.2 + 0.4j, 2.0j])
    v = np.array([1.0, 0.5j, -0.7])
    f = ola.fidelity(u, v)
    assert abs(ola.fidelity(np.exp(0.77j) * u, -3.0 * v) - f) < 1e-15
    assert 0.0 < f < 1.0


def test_gradient_descent_closed_form_quadratic():
    """C(theta) = 1/2 sum_k a_k theta_k^2 has gradient a * theta, so gradient
    descent gives theta_t = (1 - eta a)^t theta_0 exactly; costs[t] must be the
    cost at thetas[t] (the iterate after t steps), for every t."""
    a = np.array([1.0, 0.5, 2.0, 0.25])
    th0 = np.array([1.0, -2.0, 0.5, 4.0])
    eta, steps = 0.25, 6
    f = lambda t: (0.5 * float(np.sum(a * t * t)), a * t)
    thetas, costs = oc.gradient_descent(th0, f, eta, steps)
    assert thetas.shape == (steps + 1, 4) and costs.shape == (steps + 1,)
    for t in range(steps + 1):
        want = (1.0 - eta * a) ** t * th0
        assert np.max(np.abs(thetas[t] - want)) < 1e-15
        assert abs(costs[t] - 0.5 * float(np.sum(a * want * want))) < 1e-14
