"""Plant plausible mistakes in copies of oracle routines (CPU only) and check
that the pins used elsewhere catch each of them."""
import math

import numpy as np

from oracle import circuit as qc
from oracle import pauli as op


def _fwht_variant(A, phase_sign=-1, transpose_gather=False):
    N = A.shape[0]
    k = np.arange(N)
    C = np.zeros((N, N), dtype=np.complex128)
    for x in range(N):
        v = A[k, k ^ x] if transpose_gather else A[k ^ x, k]
        w = op.walsh_hadamard(v)
        ny = np.bitwise_count(np.uint64(x) & k.astype(np.uint64)).astype(np.int64) % 4
        C[x, :] = (phase_sign * 1j) ** ny * w / N
    return C


def test_pins_catch_fwht_mistakes():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    ref = op.decompose_bruteforce(A)
    assert np.max(np.abs(_fwht_variant(A) - ref)) < 1e-14
    assert np.max(np.abs(_fwht_variant(A, phase_sign=+1) - ref)) > 1e-3       # wrong phase sign
    assert np.max(np.abs(_fwht_variant(A, transpose_gather=True) - ref)) > 1e-3  # transposed operand


def test_pins_catch_hadamard_mistakes():
    """S instead of S^dagger flips the imaginary part; a missing final H gives
    a constant; both differ from the dense overlap."""
    n, layers = 2, 1
    th = np.array([0.3, 1.1])
    x = qc.ansatz_state(th, n, layers)
    l, m = (0b01, 0b00), (0b01, 0b01)
    U = op.pauli_string_matrix(*l, n).conj().T @ op.pauli_string_matrix(*m, n)
    want = np.vdot(x, U @ x).imag

    def circuit(sdg_phase, final_h=True):
        psi = qc._start(n)
        psi = qc.apply_ansatz(psi, th, n, layers, "cz")
        psi = qc.apply_controlled_pauli(psi, n, *m, n)
        psi = qc.apply_controlled_pauli(psi, n, *l, n)
        psi = qc.apply_1q(psi, n, np.diag([1.0, sdg_phase]).astype(complex))
        if final_h:
            psi = qc.apply_1q(psi, n, qc.H2)
        return qc.z_expectation(psi, n)

    assert abs(circuit(-1j) - want) < 1e-14
    assert abs(circuit(+1j) - want) > 0.1
    assert abs(circuit(-1j, final_h=False) - want) > 0.1


def test_pins_catch_ry_sign_mistake():
    """RY with the sine on the wrong side differs from the dense Kronecker pin."""
    n = 2
    psi = np.zeros(4, complex)
    psi[0] = 1
    t = 0.7
    good = qc.apply_1q(psi, 0, qc.ry(t))
    bad = qc.apply_1q(psi, 0, qc.ry(t).T)
    c, s = math.cos(t / 2), math.sin(t / 2)
    want = np.kron(np.eye(2), np.array([[c, -s], [s, c]]))[:, 0]
    assert np.allclose(good, want) and not np.allclose(bad, want)


def test_pins_catch_ccx_control_mistake(monkeypatch):
    """A doubly controlled X that ignores its ladder control (X on the target
    wherever the ancilla is 1), or one with control and target of the ladder
    gate swapped, changes the controlled V(theta) of the gamma circuit; the
    dense-overlap pin of the CNOT-ladder gamma circuit sees both.  (Dropping
    the ancilla control instead is harmless: the ancilla-0 half stays |0>,
    which a CNOT leaves alone.)"""
    n, layers = 3, 2
    th = np.array([0.4, 1.3, -0.8, 2.1, 0.2, -1.7])
    b = np.full(1 << n, 1 / math.sqrt(1 << n))
    x = qc.ansatz_state(th, n, layers, "cnot")
    l = (0b101, 0b011)
    want = np.vdot(b, op.pauli_string_matrix(*l, n) @ x)
    assert abs(qc.gamma_term(th, n, layers, "cnot", l) - want) < 1e-14

    good = qc._apply_ccx

    def ccx_ancilla_only(psi, c1, c2, t):
        return qc.apply_controlled_1q(psi, c1, t, op.X2)

    def ccx_swapped(psi, c1, c2, t):
        return good(psi, c1, t, c2)

    for bad in (ccx_ancilla_only, ccx_swapped):
        monkeypatch.setattr(qc, "_apply_ccx", bad)
        assert abs(qc.gamma_term(th, n, layers, "cnot", l) - want) > 1e-3


def test_pins_catch_fidelity_mistakes():
    """|<u|v>| without the square, or without the conjugate of u, fails the
    hand values the fidelity pin uses."""
    from oracle import linalg as ola

    no_square = lambda u, v: float(abs(np.vdot(ola.normalized(u), ola.normalized(v))))
    no_conj = lambda u, v: float(abs(np.sum(ola.normalized(u) * ola.normalized(v))) ** 2)
    assert abs(ola.fidelity([1.0, 0.0], [1.0, 1.0]) - 0.5) < 1e-15
    assert abs(no_square([1.0, 0.0], [1.0, 1.0]) - 0.5) > 0.1
    assert abs(ola.fidelity([1.0, 1j], [1.0, -1j])) < 1e-15
    assert abs(no_conj([1.0, 1j], [1.0, -1j])) > 0.5


def test_pins_catch_gradient_descent_alignment_mistake():
    """Recording the cost after the update (costs[t] = C(theta_{t+1})) breaks
    the closed-form quadratic pin."""
    from oracle import cost as oc

    def shifted(theta0, fn, eta, steps):
        th = np.asarray(theta0, dtype=np.float64).copy()
        thetas, costs = [th.copy()], []
        for _ in range(steps):
            _, g = fn(th)
            th = th - eta * g
            thetas.append(th.copy())
            costs.append(fn(th)[0])
        costs.append(fn(th)[0])
        return np.array(thetas), np.array(costs)

    a = np.array([1.0, 0.5])
    th0 = np.array([1.0, -2.0])
    f = lambda t: (0.5 * float(np.sum(a * t * t)), a * t)
    for gd, ok in ((oc.gradient_descent, True), (shifted, False)):
        thetas, costs = gd(th0, f, 0.25, 3)
        match = all(abs(costs[t] - 0.5 * np.sum(a * ((1 - 0.25 * a) ** t * th0) ** 2)) < 1e-14
                    for t in range(4))
        assert match == ok


def test_pins_catch_global_count_mistake(monkeypatch):
    """A global count of 2L^2 + L (one circuit per gamma term) disagrees with
    the circuits the oracle's enumeration runs."""
    calls = {"n": 0}

    def counted(*a, **k):
        calls["n"] += 1
        return 0.0

    for name in ("beta_circuit", "gamma_circuit"):
        monkeypatch.setattr(qc, name, counted)
    n, L = 3, 8
    qc.terms(np.zeros(n), n, 1, "cz", list(range(L)), list(range(L)), "global")
    assert calls["n"] == op.circuits_per_evaluation(n, L, "global")
    assert calls["n"] != 2 * L * L + L
