"""Pins of the oracle's Pauli decomposition and pruning (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import linalg as ola
from oracle import pauli as op
from workloads import gaussian_rhs, random_symmetric, toeplitz


def _rand_complex(n, seed):
    rng = np.random.default_rng(seed)
    N = 1 << n
    return rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_fwht_matches_bruteforce_trace(n):
    """Brute force Tr(P^dagger A)/N with explicit Kronecker products (Eq. (5))."""
    A = _rand_complex(n, 10 + n)
    assert np.max(np.abs(op.decompose_fwht(A) - op.decompose_bruteforce(A))) < 1e-14


def test_pauli_orthogonality_eq5():
    """Tr(sigma_l^dagger sigma_l') = N delta_ll' (Eq. (5)), n = 3."""
    n, N = 3, 8
    mats = [op.pauli_string_matrix(x, z, n) for x in range(N) for z in range(N)]
    G = np.array([[np.trace(a.conj().T @ b) for b in mats] for a in mats])
    assert np.allclose(G, N * np.eye(N * N), atol=1e-14)


def test_string_convention_y_is_ixz():
    """P_{x,z} = i^{|x&z|} X^x Z^z, qubit q <-> bit q (single-qubit check and a 2-qubit one)."""
    X = op.pauli_string_matrix(1, 0, 1)
    Z = op.pauli_string_matrix(0, 1, 1)
    assert np.allclose(op.pauli_string_matrix(1, 1, 1), 1j * X @ Z)
    # 2 qubits: x = 0b01 (X on qubit 0), z = 0b10 (Z on qubit 1) -> Z (x) X
    assert np.allclose(op.pauli_string_matrix(0b01, 0b10, 2), np.kron(op.Z2, op.X2))
    assert op.pauli_label(0b01, 0b10, 2) == "ZX"


@pytest.mark.parametrize("n,seed", [(3, 0), (6, 1)])
def test_parseval(n, seed):
    """N * sum |c|^2 = ||A||_F^2 (consequence of Eq. (5))."""
    A = _rand_complex(n, seed)
    C = op.decompose_fwht(A)
    N = 1 << n
    assert abs(N * np.sum(np.abs(C) ** 2) - np.linalg.norm(A) ** 2) < 1e-10 * np.linalg.norm(A) ** 2


def test_full_reconstruction_and_frobenius_closed_form():
    """sum_l c_l P_l = A, and ||A - A_tilde||_F = sqrt(N sum_dropped |c|^2)."""
    n = 4
    A = random_symmetric(n, seed=3)
    C = op.decompose_fwht(A)
    flat = np.arange(C.size)
    c, x, z = op.kept_terms(C, flat)
    assert np.max(np.abs(op.reconstruct(c, x, z, n) - A)) < 1e-13
    keep = op.select_top(C, 40)
    c, x, z = op.kept_terms(C, keep)
    At = op.reconstruct(c, x, z, n)
    direct = np.linalg.norm(A - At) / np.linalg.norm(A)
    assert abs(op.frobenius_error(C, keep, A) - direct) < 1e-13


def test_real_symmetric_parity_structure():
    """Real symmetric A: strings with an odd number of Y vanish, the rest are real."""
    n = 4
    A = random_symmetric(n, seed=5)
    C = op.decompose_fwht(A)
    N = 1 << n
    for x in range(N):
        for z in range(N):
            ny = bin(x & z).count("1")
            if ny % 2:
                assert abs(C[x, z]) < 1e-15
            else:
                assert abs(C[x, z].imag) < 1e-15


def toeplitz_closed_form(n, a, b):
    """Pauli coefficients of tridiag(b, a, b) written out from the structure of
    the +1 / -1 shifts: identity coefficient a; for level k = 0..n-1 the
    x-mask is 2^{k+1}-1 (the bits that flip when k trailing ones carry), and
    every even-weight z inside it has coefficient b 2^{-k} (-1)^{|z|/2 + z_k}."""
    N = 1 << n
    C = np.zeros((N, N))
    C[0, 0] = a
    for k in range(n):
        x = (1 << (k + 1)) - 1
        for z in range(N):
            if z & ~x:
                continue
            w = bin(z).count("1")
            if w % 2 == 0:
                C[x, z] = b * 2.0 ** (-k) * (-1) ** (w // 2 + ((z >> k) & 1))
    return C


@pytest.mark.parametrize("n,b", [(4, -0.45), (6, -1.0 / 3.0), (10, -0.45)])
def test_toeplitz_closed_form_bit_exact(n, b):
    C = op.decompose_fwht(toeplitz(n, 1.0, b))
    assert np.array_equal(C.imag, np.zeros_like(C.imag))
    assert np.array_equal(C.real, toeplitz_closed_form(n, 1.0, b))
    # the family has exactly 2^n nonzero strings before pruning (Section II-B)
    assert np.count_nonzero(C) == 1 << n


def test_paper_pruning_table(golden_dir):
    """L(tau) and epsilon_F of Section III-B for n = 10, a = 1, off-diagonal -1/3."""
    g = json.load(open(os.path.join(golden_dir, "pruning_toeplitz_n10.json")))
    n = g["system"]["n"]
    A = toeplitz(n, g["system"]["a"], g["system"]["off_diagonal"])
    C = op.decompose_fwht(A)
    Ls = [len(op.select_tau(C, t)) for t in g["tau"]]
    assert Ls == g["L_retained"]
    for L, pct in g["frobenius_error_percent"].items():
        keep = op.select_top(C, int(L))
        assert round(100 * op.frobenius_error(C, keep, A), 2) == pct
    for L, count in g["circuits_per_iteration"].items():
        assert op.circuits_per_evaluation(n, int(L), "local") == count


@pytest.mark.slow
def test_paper_median_solution_error_loose(golden_dir):
    """Median relative solution error over 64 Gaussian RHS (Section III-B).
    The paper's seed is not given: compared within 1 percentage point."""
    g = json.load(open(os.path.join(golden_dir, "pruning_toeplitz_n10.json")))
    n = 10
    A = toeplitz(n, 1.0, -1.0 / 3.0)
    C = op.decompose_fwht(A)
    rhs = gaussian_rhs(1 << n, 64, seed=0)
    for L, pct in g["median_solution_error_percent"].items():
        keep = op.select_top(C, int(L))
        At = op.reconstruct(*op.kept_terms(C, keep), n).real
        med = 100 * np.median(ola.relative_solution_errors(A, At, rhs))
        assert abs(med - pct) < 1.0, (L, med, pct)
        # the perturbation bound of Eq. (6) holds whenever it applies
        bound = ola.perturbation_bound(A, At)
        errs = ola.relative_solution_errors(A, At, rhs)
        assert np.all(errs <= bound + 1e-12)


def test_resource_rule(golden_dir):
    """L_post = min(2^n, 64) at tau = 0.01 (Fig. 2 caption, Section II-E)."""
    g = json.load(open(os.path.join(golden_dir, "resources_toeplitz.json")))
    fam = g["family"]
    for n, lpre, lpost in zip(g["n"], g["L_pre"], g["L_post"]):
        C = op.decompose_fwht(toeplitz(n, fam["a"], fam["off_diagonal"]))
        assert np.count_nonzero(np.abs(C) > 0) == lpre
        assert len(op.select_tau(C, fam["tau"])) == lpost


def test_selection_order_and_ties():
    """Ranking: |c| descending, then flat index ascending; tau is strict."""
    C = np.zeros((4, 4), dtype=complex)
    C[0, 0] = 1.0
    C[1, 0] = -0.5
    C[0, 1] = 0.5j       # ties with C[1,0] in magnitude, smaller flat index (1 < 4)
    C[3, 3] = 0.25
    C[2, 2] = 0.25 + 0j  # ties with C[3,3], flat 10 < 15
    assert list(op.select_top(C, 5)) == [0, 1, 4, 10, 15]
    assert list(op.select_tau(C, 0.25)) == [0, 1, 4]
    assert list(op.select_tau(C, 0.2499)) == [0, 1, 4, 10, 15]


@pytest.mark.parametrize("kind,n,L", [("global", 3, 8), ("local", 3, 8), ("global", 2, 3), ("local", 2, 3)])
def test_circuit_count_equals_enumerated_circuits(monkeypatch, kind, n, L):
    """The count the oracle reports equals the number of Hadamard-test
    circuits its own term enumeration runs (each complex term is a real and
    an imaginary circuit): global 2(L^2 + L) -- 144 at n = 3, L = 8 --,
    local 2(n+1)L^2 (Section II-B after Eq. (4))."""
    from oracle import circuit as qc

    calls = {"n": 0}
    for name in ("beta_circuit", "delta_circuit", "gamma_circuit"):
        def counted(*a, _f=getattr(qc, name), **k):
            calls["n"] += 1
            return 0.0
        monkeypatch.setattr(qc, name, counted)
    xs = list(range(L))
    qc.terms(np.zeros(n), n, 1, "cz", xs, xs, kind)
    assert calls["n"] == op.circuits_per_evaluation(n, L, kind)
    if (kind, n, L) == ("global", 3, 8):
        assert calls["n"] == 144
