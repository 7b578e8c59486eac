"""Pauli decomposition and pruning -- oracle (test infrastructure only).

Paper: Section II-B.  A matrix of dimension N = 2^n is written as a linear
combination of Pauli strings, c_l = Tr(sigma_l^dagger A) / N, using the
orthogonality Tr(sigma_l^dagger sigma_l') = N delta (Eq. (5)).  Pruning keeps
every term with |c_l| > tau (Section II-B, Algorithm 1 Step 2) or the L
largest-magnitude terms (Section III-B, "magnitude-ranked").

Conventions (this project's reading, shared with the GPU path by
specification, not by code):
  * basis index bit q <-> qubit q;
  * a string is a pair of n-bit masks (x, z):
        P_{x,z} = i^{popcount(x & z)} X^x Z^z = (tensor over q of sigma_q),
    sigma_q = I, X, Z, Y for (x_q, z_q) = (0,0), (1,0), (0,1), (1,1);
  * the flat index of a string is x * N + z;
  * ranking key: |c| descending (|c| = hypot(re, im) in FP64), then flat
    index ascending.

Pins: brute force vs FWHT (n <= 5), Parseval, the Toeplitz closed form,
the paper's L(tau) and epsilon_F table (Section III-B).
"""
from __future__ import annotations

import numpy as np

I2 = np.array([[1, 0], [0, 1]], dtype=np.complex128)
X2 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z2 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def pauli_factor(xb: int, zb: int) -> np.ndarray:
    """Single-qubit Pauli for one bit pair of the (x, z) masks."""
    return {(0, 0): I2, (1, 0): X2, (0, 1): Z2, (1, 1): Y2}[(xb, zb)]


def pauli_string_matrix(x: int, z: int, n: int) -> np.ndarray:
    """Dense 2^n x 2^n matrix of the string (x, z), as a Kronecker product.

    Qubit n-1 is the leftmost factor because it is the most significant bit
    of the basis index.
    """
    M = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(n)):
        M = np.kron(M, pauli_factor((x >> q) & 1, (z >> q) & 1))
    return M


def pauli_label(x: int, z: int, n: int) -> str:
    """Text label, qubit n-1 on the left (e.g. 'IXYZ')."""
    s = {(0, 0): "I", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}
    return "".join(s[((x >> q) & 1, (z >> q) & 1)] for q in reversed(range(n)))


def decompose_bruteforce(A: np.ndarray) -> np.ndarray:
    """c[x, z] = Tr(P_{x,z}^dagger A) / N for every string (Eq. (5)).

    Explicit Kronecker products and traces; O(16^n N) work, use for n <= 5.
    """
    N = A.shape[0]
    n = N.bit_length() - 1
    C = np.zeros((N, N), dtype=np.complex128)
    for x in range(N):
        for z in range(N):
            P = pauli_string_matrix(x, z, n)
            C[x, z] = np.trace(P.conj().T @ A) / N
    return C


def walsh_hadamard(v: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform: W[z] = sum_k (-1)^{popcount(z&k)} v[k].

    Plain radix-2 butterflies, one stage per bit: at stage h the pairs
    (k, k + h) with bit h of k clear become (a + b, a - b).
    """
    v = np.array(v, dtype=np.complex128, copy=True)
    N = v.shape[0]
    h = 1
    while h < N:
        blocks = v.reshape(N // (2 * h), 2, h)
        a = blocks[:, 0, :].copy()
        b = blocks[:, 1, :].copy()
        blocks[:, 0, :] = a + b
        blocks[:, 1, :] = a - b
        v = blocks.reshape(N)
        h *= 2
    return v


def decompose_fwht(A: np.ndarray) -> np.ndarray:
    """All 4^n coefficients through one Walsh-Hadamard transform per x-mask.

    Tr(P_{x,z}^dagger A) = (-i)^{popcount(x&z)} sum_k (-1)^{popcount(z&k)} A[k^x, k],
    because P_{x,z}^dagger = (-i)^{|x&z|} Z^z X^x, <k| Z^z = (-1)^{z.k} <k| and
    <k| X^x = <k^x|.  So for each x: gather v[k] = A[k^x, k], transform over k,
    divide by N and multiply by the phase (Section II-B; the FWHT route the
    paper adopts).  Returns C[x, z].
    """
    N = A.shape[0]
    n = N.bit_length() - 1
    assert N == 1 << n
    k = np.arange(N)
    C = np.zeros((N, N), dtype=np.complex128)
    for x in range(N):
        w = walsh_hadamard(A[k ^ x, k])
        ny = np.bitwise_count(np.uint64(x) & k.astype(np.uint64)).astype(np.int64) % 4
        C[x, :] = np.array([1, -1j, -1, 1j])[ny] * w / N
    return C


def magnitudes(C: np.ndarray) -> np.ndarray:
    """|c| = hypot(re, im) in FP64, flattened in x*N + z order."""
    return np.abs(C).ravel()


def rank_order(C: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Order flat indices by (|c| descending, index ascending)."""
    mag = magnitudes(C)[idx]
    return idx[np.lexsort((idx, -mag))]


def select_tau(C: np.ndarray, tau: float) -> np.ndarray:
    """Flat indices with |c| > tau (strict), in ranking order (Alg. 1 Step 2)."""
    mag = magnitudes(C)
    idx = np.nonzero(mag > tau)[0]
    return rank_order(C, idx)


def select_top(C: np.ndarray, L: int) -> np.ndarray:
    """The L highest-ranked flat indices (Section III-B)."""
    idx = np.arange(C.size)
    return rank_order(C, idx)[:L]


def split_index(flat: np.ndarray, n: int):
    """Flat index x*N + z -> (x, z) masks."""
    N = 1 << n
    flat = np.asarray(flat, dtype=np.int64)
    return flat // N, flat % N


def kept_terms(C: np.ndarray, flat: np.ndarray):
    """(coeffs, x, z) of the kept strings, in the order given."""
    n = C.shape[0].bit_length() - 1
    x, z = split_index(flat, n)
    return C.ravel()[flat], x, z


def frobenius_error(C: np.ndarray, flat_kept: np.ndarray, A: np.ndarray) -> float:
    """Relative matrix error of the pruned sum.

    By Eq. (5) the strings are orthogonal with squared norm N, so
    ||A - A_tilde||_F^2 = N * sum over dropped strings of |c|^2; this returns
    that square root divided by ||A||_F.
    """
    N = A.shape[0]
    mask = np.ones(C.size, dtype=bool)
    mask[flat_kept] = False
    dropped = np.sum(np.abs(C.ravel()[mask]) ** 2)
    return float(np.sqrt(N * dropped) / np.linalg.norm(A))


def reconstruct(coeffs, xs, zs, n: int) -> np.ndarray:
    """A_tilde = sum_l c_l P_l as a dense matrix (Eq. (3))."""
    N = 1 << n
    M = np.zeros((N, N), dtype=np.complex128)
    for c, x, z in zip(coeffs, xs, zs):
        M += c * pauli_string_matrix(int(x), int(z), n)
    return M


def circuits_per_evaluation(n: int, L: int, kind: str = "local") -> int:
    """Hadamard-test circuits per cost evaluation.

    Local cost: n*L^2 numerator + L^2 denominator expectation values, each
    with a real and an imaginary circuit: 2(n+1)L^2 (Section II-B, after
    Eq. (4)).  Global cost: L^2 denominator + L overlap terms, 2(L^2 + L).
    """
    if kind == "local":
        return 2 * (n + 1) * L * L
    return 2 * (L * L + L)
