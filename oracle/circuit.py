"""Gate-by-gate Hadamard-test circuits -- oracle (test infrastructure only).

Paper: Section II-A (VQLS, Hadamard tests), Section II-C (circuit body:
ansatz, two controlled Pauli strings, controlled Z_j, ancilla preparation and
measurement) and Eq. (4) (the terms of the expanded cost).

Register: n system qubits (bits 0..n-1 of the basis index) and one ancilla,
bit n.  Every gate is an explicit 2x2 matrix applied to the 2^(n+1)-amplitude
state vector; nothing is fused or reordered.

Ansatz V(theta) (this project's reading of Section II-C / Section III-A):
``layers`` layers; layer l applies RY(theta[l*n + q]) on every qubit q, then
an entangling ladder on (q, q+1), q = 0..n-2: CZ gates ("cz") or CNOT with
control q and target q+1 ("cnot").  RY(t) = [[cos t/2, -sin t/2],
[sin t/2, cos t/2]].

State preparation U_b (U_b|0> = |b>):
  * b = |+>^n: U_b = H on every system qubit;
  * a real vector b: U_b = s (I - 2 w w^T / (w^T w)), w = e_0 - s b,
    s = -1 if b_0 > 0 else +1 (a Householder reflector; U_b = U_b^dagger).

Circuits (ancilla a = qubit n; A_l^dagger = A_l for Pauli strings):
  beta_lm  = <x|A_l^dagger A_m|x>:
      H(a); V; C-A_m; C-A_l; [S^dagger(a)]; H(a)
  delta^j_lm = <x|A_l^dagger U_b Z_j U_b^dagger A_m|x>   (local cost):
      H(a); V; C-A_m; U_b^dagger; CZ(a, j); U_b; C-A_l; [S^dagger(a)]; H(a)
  gamma_l  = <b|A_l|x> = <0|U_b^dagger A_l V|0>          (global cost):
      H(a); C-V; C-A_l; C-U_b^dagger; [S^dagger(a)]; H(a)
and <Z_a> = P(a=0) - P(a=1) equals the real part of the overlap, or its
imaginary part when S^dagger is applied before the final H.

Pins: the ansatz against a dense product of Kronecker matrices, every circuit
against the overlap computed with dense matrices, the theta = 0 case by
hand, and the beta invariants (tests/test_oracle_circuit.py).
"""
from __future__ import annotations

import math

import numpy as np

from .pauli import X2, Y2, Z2, pauli_factor

H2 = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
SDG2 = np.array([[1, 0], [0, -1j]], dtype=np.complex128)


def ry(t: float) -> np.ndarray:
    c, s = math.cos(t / 2.0), math.sin(t / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


# ---------------------------------------------------------------- primitives

def apply_1q(psi: np.ndarray, q: int, U: np.ndarray) -> np.ndarray:
    """Apply the 2x2 matrix U on qubit q."""
    nb = psi.shape[0].bit_length() - 1
    v = psi.reshape(1 << (nb - q - 1), 2, 1 << q)
    out = np.empty_like(v)
    out[:, 0, :] = U[0, 0] * v[:, 0, :] + U[0, 1] * v[:, 1, :]
    out[:, 1, :] = U[1, 0] * v[:, 0, :] + U[1, 1] * v[:, 1, :]
    return out.reshape(-1)


def _bit_set(nb: int, q: int) -> np.ndarray:
    return ((np.arange(1 << nb) >> q) & 1).astype(bool)


def apply_controlled_1q(psi: np.ndarray, ctrl: int, q: int, U: np.ndarray) -> np.ndarray:
    """Apply U on qubit q where qubit ctrl is 1 (ctrl != q)."""
    assert ctrl != q
    nb = psi.shape[0].bit_length() - 1
    full = apply_1q(psi, q, U)
    out = psi.copy()
    m = _bit_set(nb, ctrl)
    out[m] = full[m]
    return out


def apply_cz(psi: np.ndarray, a: int, b: int) -> np.ndarray:
    nb = psi.shape[0].bit_length() - 1
    m = _bit_set(nb, a) & _bit_set(nb, b)
    out = psi.copy()
    out[m] = -out[m]
    return out


def apply_cnot(psi: np.ndarray, ctrl: int, tgt: int) -> np.ndarray:
    return apply_controlled_1q(psi, ctrl, tgt, X2)


def apply_dense_system(psi: np.ndarray, n: int, M: np.ndarray, ctrl: int | None = None) -> np.ndarray:
    """Apply a dense 2^n x 2^n matrix on the system register (bits 0..n-1),
    optionally only where the ancilla (bit n) is 1."""
    N = 1 << n
    v = psi.reshape(2, N)
    out = v.copy()
    if ctrl is None:
        out[0] = M @ v[0]
        out[1] = M @ v[1]
    else:
        assert ctrl == n
        out[1] = M @ v[1]
    return out.reshape(-1)


# ---------------------------------------------------------------- blocks

def ansatz_gates(n: int, layers: int, entangler: str = "cz"):
    """Gate list of V(theta): ('ry', q, k) with angle index k, or (ent, q, q+1)."""
    gates = []
    for l in range(layers):
        for q in range(n):
            gates.append(("ry", q, l * n + q))
        for q in range(n - 1):
            gates.append((entangler, q, q + 1))
    return gates


def apply_ansatz(psi, theta, n, layers, entangler="cz", ctrl=None):
    for g in ansatz_gates(n, layers, entangler):
        kind = g[0]
        if kind == "ry":
            U = ry(float(theta[g[2]]))
            psi = apply_1q(psi, g[1], U) if ctrl is None else apply_controlled_1q(psi, ctrl, g[1], U)
        elif kind == "cz":
            if ctrl is None:
                psi = apply_cz(psi, g[1], g[2])
            else:
                psi = _apply_ccz(psi, ctrl, g[1], g[2])
        elif kind == "cnot":
            if ctrl is None:
                psi = apply_cnot(psi, g[1], g[2])
            else:
                psi = _apply_ccx(psi, ctrl, g[1], g[2])
        else:
            raise ValueError(kind)
    return psi


def _apply_ccz(psi, c1, c2, c3):
    nb = psi.shape[0].bit_length() - 1
    m = _bit_set(nb, c1) & _bit_set(nb, c2) & _bit_set(nb, c3)
    out = psi.copy()
    out[m] = -out[m]
    return out


def _apply_ccx(psi, c1, c2, t):
    nb = psi.shape[0].bit_length() - 1
    full = apply_1q(psi, t, X2)
    m = _bit_set(nb, c1) & _bit_set(nb, c2)
    out = psi.copy()
    out[m] = full[m]
    return out


def apply_controlled_pauli(psi, ctrl, x, z, n):
    """Controlled Pauli string: one controlled single-qubit Pauli per qubit."""
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb or zb:
            psi = apply_controlled_1q(psi, ctrl, q, pauli_factor(xb, zb))
    return psi


def householder_ub(b: np.ndarray) -> np.ndarray:
    """Dense U_b for a real normalised vector b (see module docstring)."""
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    s = -1.0 if b[0] > 0 else 1.0
    w = -s * b.copy()
    w[0] += 1.0
    R = np.eye(N) - 2.0 * np.outer(w, w) / np.dot(w, w)
    return s * R


def apply_ub(psi, n, b_kind, b=None, dagger=False, ctrl=None):
    """U_b (or U_b^dagger) on the system register."""
    if b_kind == "plus":
        for q in range(n):
            psi = apply_1q(psi, q, H2) if ctrl is None else apply_controlled_1q(psi, ctrl, q, H2)
        return psi
    U = householder_ub(b)
    if dagger:
        U = U.conj().T
    return apply_dense_system(psi, n, U.astype(np.complex128), ctrl=ctrl)


def z_expectation(psi: np.ndarray, q: int) -> float:
    """<Z_q> = P(bit q = 0) - P(bit q = 1)."""
    nb = psi.shape[0].bit_length() - 1
    m = _bit_set(nb, q)
    p = np.abs(psi) ** 2
    return float(p[~m].sum() - p[m].sum())


# ---------------------------------------------------------------- circuits

def _start(n):
    psi = np.zeros(1 << (n + 1), dtype=np.complex128)
    psi[0] = 1.0
    return apply_1q(psi, n, H2)


def _finish(psi, n, imag):
    if imag:
        psi = apply_1q(psi, n, SDG2)
    psi = apply_1q(psi, n, H2)
    return z_expectation(psi, n)


def beta_circuit(theta, n, layers, ent, l_xz, m_xz, imag):
    """<Z_a> of the beta_lm circuit (real or imaginary part)."""
    a = n
    psi = _start(n)
    psi = apply_ansatz(psi, theta, n, layers, ent)
    psi = apply_controlled_pauli(psi, a, m_xz[0], m_xz[1], n)
    psi = apply_controlled_pauli(psi, a, l_xz[0], l_xz[1], n)
    return _finish(psi, n, imag)


def delta_circuit(theta, n, layers, ent, l_xz, m_xz, j, imag, b_kind="plus", b=None):
    """<Z_a> of the delta^j_lm circuit (local cost numerator, Z_j on qubit j)."""
    a = n
    psi = _start(n)
    psi = apply_ansatz(psi, theta, n, layers, ent)
    psi = apply_controlled_pauli(psi, a, m_xz[0], m_xz[1], n)
    psi = apply_ub(psi, n, b_kind, b, dagger=True)
    psi = apply_cz(psi, a, j)
    psi = apply_ub(psi, n, b_kind, b, dagger=False)
    psi = apply_controlled_pauli(psi, a, l_xz[0], l_xz[1], n)
    return _finish(psi, n, imag)


def gamma_circuit(theta, n, layers, ent, l_xz, imag, b_kind="plus", b=None):
    """<Z_a> of the gamma_l circuit (global cost overlap <b|A_l|x>)."""
    a = n
    psi = _start(n)
    psi = apply_ansatz(psi, theta, n, layers, ent, ctrl=a)
    psi = apply_controlled_pauli(psi, a, l_xz[0], l_xz[1], n)
    psi = apply_ub(psi, n, b_kind, b, dagger=True, ctrl=a)
    return _finish(psi, n, imag)


def beta_term(theta, n, layers, ent, l_xz, m_xz):
    return complex(beta_circuit(theta, n, layers, ent, l_xz, m_xz, False),
                   beta_circuit(theta, n, layers, ent, l_xz, m_xz, True))


def delta_term(theta, n, layers, ent, l_xz, m_xz, j, b_kind="plus", b=None):
    return complex(delta_circuit(theta, n, layers, ent, l_xz, m_xz, j, False, b_kind, b),
                   delta_circuit(theta, n, layers, ent, l_xz, m_xz, j, True, b_kind, b))


def gamma_term(theta, n, layers, ent, l_xz, b_kind="plus", b=None):
    return complex(gamma_circuit(theta, n, layers, ent, l_xz, False, b_kind, b),
                   gamma_circuit(theta, n, layers, ent, l_xz, True, b_kind, b))


def terms(theta, n, layers, ent, xs, zs, kind, b_kind="plus", b=None):
    """Every term of one cost evaluation, one circuit pair per term.

    Returns (beta[L, L], other) with other = gamma[L] (kind 'global') or
    delta[n, L, L] (kind 'local').
    """
    L = len(xs)
    strings = [(int(xs[i]), int(zs[i])) for i in range(L)]
    beta = np.zeros((L, L), dtype=np.complex128)
    for l in range(L):
        for m in range(L):
            beta[l, m] = beta_term(theta, n, layers, ent, strings[l], strings[m])
    if kind == "global":
        other = np.array([gamma_term(theta, n, layers, ent, strings[l], b_kind, b) for l in range(L)])
    else:
        other = np.zeros((n, L, L), dtype=np.complex128)
        for j in range(n):
            for l in range(L):
                for m in range(L):
                    other[j, l, m] = delta_term(theta, n, layers, ent, strings[l], strings[m], j, b_kind, b)
    return beta, other


def ansatz_state(theta, n, layers, ent="cz") -> np.ndarray:
    """|x(theta)> = V(theta)|0> on the n system qubits (gate by gate)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return apply_ansatz(psi, theta, n, layers, ent)


def plus_vector(n: int) -> np.ndarray:
    """|+>^n = U_b|0> for U_b = H^n."""
    return np.full(1 << n, 1.0 / math.sqrt(1 << n), dtype=np.complex128)
