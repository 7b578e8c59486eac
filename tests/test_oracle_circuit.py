"""Pins of the oracle's gate-by-gate Hadamard-test circuits (CPU only).

Every circuit is checked against the overlap it should measure, computed with
dense matrices built from Kronecker products (no gate-application code), plus
the theta = 0 case worked by hand and the invariants of beta.
"""
import math

import numpy as np
import pytest

from oracle import circuit as qc
from oracle import pauli as op
from workloads import random_unit_vector, theta_uniform, toeplitz


def ry_dense(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -s], [s, c]])


def ansatz_unitary_dense(theta, n, layers, ent):
    """V(theta) as a product of layer matrices: Kronecker product of RYs, then
    the ladder as a diagonal (CZ) or a permutation matrix (CNOT)."""
    N = 1 << n
    idx = np.arange(N)
    V = np.eye(N)
    for l in range(layers):
        R = np.ones((1, 1))
        for q in reversed(range(n)):
            R = np.kron(R, ry_dense(theta[l * n + q]))
        E = np.eye(N)
        for q in range(n - 1):
            if ent == "cz":
                d = np.where(((idx >> q) & 1) & ((idx >> (q + 1)) & 1), -1.0, 1.0)
                G = np.diag(d)
            else:
                G = np.zeros((N, N))
                tgt = idx ^ (((idx >> q) & 1) << (q + 1))
                G[tgt, idx] = 1.0
            E = G @ E
        V = E @ R @ V
    return V


@pytest.mark.parametrize("ent", ["cz", "cnot"])
@pytest.mark.parametrize("n,layers", [(3, 2), (4, 3)])
def test_ansatz_matches_dense_product(n, layers, ent):
    th = theta_uniform(n * layers, seed=7)
    x = qc.ansatz_state(th, n, layers, ent)
    ref = ansatz_unitary_dense(th, n, layers, ent)[:, 0]
    assert np.max(np.abs(x - ref)) < 1e-14


def _strings(n, seed, L):
    rng = np.random.default_rng(seed)
    N = 1 << n
    return [(int(rng.integers(N)), int(rng.integers(N))) for _ in range(L)]


@pytest.mark.parametrize("ent", ["cz", "cnot"])
def test_beta_circuit_equals_dense_overlap(ent):
    n, layers = 3, 2
    th = theta_uniform(n * layers, seed=1)
    x = ansatz_unitary_dense(th, n, layers, ent)[:, 0]
    for (lx, lz), (mx, mz) in zip(_strings(n, 2, 6), _strings(n, 3, 6)):
        U = op.pauli_string_matrix(lx, lz, n).conj().T @ op.pauli_string_matrix(mx, mz, n)
        want = np.vdot(x, U @ x)
        got = qc.beta_term(th, n, layers, ent, (lx, lz), (mx, mz))
        assert abs(got - want) < 1e-14


@pytest.mark.parametrize("b_kind", ["plus", "vector"])
def test_delta_circuit_equals_dense_overlap(b_kind):
    n, layers = 3, 2
    N = 1 << n
    th = theta_uniform(n * layers, seed=4)
    b = random_unit_vector(N, seed=9) if b_kind == "vector" else None
    x = ansatz_unitary_dense(th, n, layers, "cz")[:, 0]
    if b_kind == "plus":
        Ub = np.ones((1, 1))
        for _ in range(n):
            Ub = np.kron(Ub, np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    else:
        Ub = qc.householder_ub(b)
        assert np.allclose(Ub[:, 0], b) and np.allclose(Ub @ Ub.T, np.eye(N))
    for j in range(n):
        Zj = np.diag(1.0 - 2.0 * ((np.arange(N) >> j) & 1))
        for (lx, lz), (mx, mz) in zip(_strings(n, 5 + j, 3), _strings(n, 8 + j, 3)):
            Pl = op.pauli_string_matrix(lx, lz, n)
            Pm = op.pauli_string_matrix(mx, mz, n)
            want = np.vdot(x, Pl.conj().T @ Ub @ Zj @ Ub.conj().T @ Pm @ x)
            got = qc.delta_term(th, n, layers, "cz", (lx, lz), (mx, mz), j, b_kind, b)
            assert abs(got - want) < 1e-14


@pytest.mark.parametrize("ent", ["cz", "cnot"])
@pytest.mark.parametrize("b_kind", ["plus", "vector"])
def test_gamma_circuit_equals_dense_overlap(b_kind, ent):
    """The gamma circuit controls V(theta) itself on the ancilla: with the
    CNOT ladder every ladder gate becomes a doubly controlled X, so this pins
    the controlled-controlled X against the dense permutation matrix."""
    n, layers = 3, 2
    N = 1 << n
    th = theta_uniform(n * layers, seed=6)
    b = random_unit_vector(N, seed=11) if b_kind == "vector" else np.full(N, 1 / math.sqrt(N))
    x = ansatz_unitary_dense(th, n, layers, ent)[:, 0]
    for lx, lz in _strings(n, 12, 8):
        want = np.vdot(b, op.pauli_string_matrix(lx, lz, n) @ x)
        got = qc.gamma_term(th, n, layers, ent, (lx, lz), b_kind, b if b_kind == "vector" else None)
        assert abs(got - want) < 1e-14


def test_theta_zero_by_hand():
    """V(0)|0> = |0>, P_{x,z}|0> = i^{|x&z|}|x>, so beta_lm = conj(i^{|l|}) i^{|m|} [x_l == x_m]."""
    n, layers = 3, 2
    th = np.zeros(n * layers)
    for (lx, lz), (mx, mz) in zip(_strings(n, 20, 10), _strings(n, 21, 10)):
        mx = lx if (lx + mx) % 3 == 0 else mx  # force some equal x-masks
        pl = 1j ** bin(lx & lz).count("1")
        pm = 1j ** bin(mx & mz).count("1")
        want = np.conj(pl) * pm * (1.0 if lx == mx else 0.0)
        got = qc.beta_term(th, n, layers, "cz", (lx, lz), (mx, mz))
        assert abs(got - want) < 1e-15


def test_beta_invariants_toeplitz():
    """beta_ll = 1, Hermitian, PSD, |beta| <= 1 and Im beta = 0 for the real
    ansatz and the (real, even-Y) strings of a real symmetric matrix."""
    n, layers = 3, 2
    C = op.decompose_fwht(toeplitz(n, 1.0, -0.4))
    keep = op.select_tau(C, 0.01)
    c, xs, zs = op.kept_terms(C, keep)
    th = theta_uniform(n * layers, seed=0)
    beta, gamma = qc.terms(th, n, layers, "cz", xs, zs, "global")
    L = len(keep)
    assert L == 8
    assert np.allclose(np.diag(beta), 1.0, atol=1e-14)
    assert np.allclose(beta, beta.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(beta)) > -1e-13
    assert np.max(np.abs(beta)) <= 1.0 + 1e-14
    assert np.max(np.abs(beta.imag)) < 1e-15


def test_hadamard_test_identity_general_unitary():
    """<Z> without / with S^dagger = Re / Im <x|U|x> for the literal circuit.
    X.Y = iZ gives a purely imaginary overlap for the real ansatz state, and
    (X x X).(Z x Z) a real one; both parts are exercised."""
    n, layers = 2, 1
    th = np.array([0.3, 1.1])
    x = qc.ansatz_state(th, n, layers)
    cases = [((0b01, 0b00), (0b01, 0b01)), ((0b11, 0b00), (0b00, 0b11))]
    seen_re = seen_im = False
    for l, m in cases:
        U = op.pauli_string_matrix(*l, n).conj().T @ op.pauli_string_matrix(*m, n)
        want = np.vdot(x, U @ x)
        re = qc.beta_circuit(th, n, layers, "cz", l, m, False)
        im = qc.beta_circuit(th, n, layers, "cz", l, m, True)
        assert abs(re - want.real) < 2e-15 and abs(im - want.imag) < 2e-15
        seen_re |= abs(want.real) > 0.05
        seen_im |= abs(want.imag) > 0.05
    assert seen_re and seen_im


def test_pool_terms_equal_serial_terms():
    """The process-pool runner of the full-size GPU parity test decodes its
    flat circuit index into the same terms as the serial enumeration."""
    import _oracle_pool

    n, layers = 3, 2
    xs = np.array([0, 1, 3, 6, 2])
    zs = np.array([0, 2, 3, 5, 7])
    th = theta_uniform(n * layers, seed=4)
    wb, wd = qc.terms(th, n, layers, "cnot", xs, zs, "local")
    gb, gd = _oracle_pool.local_terms(n, layers, "cnot", xs, zs, th, procs=2)
    assert np.array_equal(gb, wb) and np.array_equal(gd, wd)
