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
