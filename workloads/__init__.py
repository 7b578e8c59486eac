"""Seeded synthetic inputs for the D-VQLS hot path.

This module is shared by the CPU oracle, the tests and the benchmark. It only
builds inputs (matrices, right-hand sides, angles); it contains none of the
method's arithmetic (no Pauli decomposition, no circuit, no cost).

Workload families (paper: arXiv 2604.14435):
  * tridiagonal Toeplitz matrices, diagonal a, off-diagonals b (super) and c
    (sub) -- Section II-D, Eq. (7);
  * a Hele-Shaw-like pressure operator: a 5-point variable-coefficient
    Laplacian on a 32x32 cell grid (the paper's Section II-D Eqs. (8)-(9)
    describe the flow; the discretisation below is this project's reading);
  * dense random symmetric matrices with N(0,1) entries;
  * the right-hand side |+>^n and seeded Gaussian / uniform right-hand sides.

All randomness comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "toeplitz",
    "plus_state",
    "random_symmetric",
    "heleshaw_like",
    "theta_uniform",
    "gaussian_rhs",
    "random_unit_vector",
    "toeplitz_family",
    "family_split",
    "CONFIGS",
]


def toeplitz(n: int, a: float, b: float, c: float | None = None) -> np.ndarray:
    """Dense 2^n x 2^n tridiagonal Toeplitz matrix (Section II-D, Eq. (7)).

    ``a`` is the main diagonal, ``b`` the super-diagonal and ``c`` the
    sub-diagonal (``c`` defaults to ``b``: the symmetric family used in the
    paper's experiments).  Returned as float64, row-major.
    """
    if c is None:
        c = b
    N = 1 << n
    A = np.zeros((N, N), dtype=np.float64)
    idx = np.arange(N)
    A[idx, idx] = a
    A[idx[:-1], idx[:-1] + 1] = b
    A[idx[:-1] + 1, idx[:-1]] = c
    return A


def plus_state(n: int) -> np.ndarray:
    """|+>^n = 2^{-n/2} (1, ..., 1): the right-hand side prepared by H^n."""
    N = 1 << n
    return np.full(N, 1.0 / math.sqrt(N), dtype=np.float64)


def random_symmetric(n: int, seed: int = 0) -> np.ndarray:
    """Dense symmetric 2^n x 2^n matrix whose entries are all N(0,1).

    Draw G ~ N(0,1) (N x N) and keep its upper triangle, mirrored.
    """
    N = 1 << n
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N))
    U = np.triu(G)
    return U + np.triu(G, 1).T


def heleshaw_like(m: int = 32, sigma: float = 0.5, seed: int = 0):
    """Hele-Shaw-like pressure system on an m x m cell grid (m a power of 2).

    Cell-centred finite volumes; unknown index u = m*i + j (j = column, in the
    low log2(m) bits).  Cell conductance k = h^3 with h = exp(N(0, sigma^2)).
    An interior face between cells p, q has conductance 2 k_p k_q / (k_p + k_q)
    (harmonic mean); a face on the Dirichlet wall has conductance 2 k_cell
    (half-cell distance).  The operator is symmetric positive definite and is
    scaled to unit spectral norm.  The source b ~ U(0,1) is normalised.

    Draw order from ``default_rng(seed)``: h (m x m normal), then b (m*m
    uniform).  Returns (A, b).
    """
    rng = np.random.default_rng(seed)
    h = np.exp(rng.normal(0.0, sigma, size=(m, m)))
    bsrc = rng.uniform(0.0, 1.0, size=m * m)
    k = h ** 3
    N = m * m
    A = np.zeros((N, N), dtype=np.float64)
    for i in range(m):
        for j in range(m):
            p = m * i + j
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < m and 0 <= jj < m:
                    q = m * ii + jj
                    t = 2.0 * k[i, j] * k[ii, jj] / (k[i, j] + k[ii, jj])
                    A[p, q] -= t
                    A[p, p] += t
                else:
                    A[p, p] += 2.0 * k[i, j]
    lam_max = np.linalg.eigvalsh(A)[-1]
    A /= lam_max
    b = bsrc / np.linalg.norm(bsrc)
    return A, b


def theta_uniform(P: int, seed: int = 0) -> np.ndarray:
    """Initial angles theta ~ U[0, 2 pi)^P from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=P)


def gaussian_rhs(N: int, count: int, seed: int = 0) -> np.ndarray:
    """``count`` normalised Gaussian right-hand sides, shape (count, N)."""
    g = np.random.default_rng(seed).standard_normal((count, N))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def random_unit_vector(N: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """A normalised random vector (real by default) for general-b inputs."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(N)
    if complex_:
        v = v + 1j * rng.standard_normal(N)
    return v / np.linalg.norm(v)


def toeplitz_family(count: int = 4096, seed: int = 0,
                    a_range=(0.8, 1.2), b_range=(-0.49, -0.1)) -> np.ndarray:
    """(a, b) pairs of the warm-start family, uniform on the given box.

    Returns shape (count, 2): column 0 = diagonal a, column 1 = off-diagonal b.
    Draw order: all a, then all b.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(*a_range, size=count)
    b = rng.uniform(*b_range, size=count)
    return np.stack([a, b], axis=1)


def family_split(count: int = 4096, n_train: int = 3584, seed: int = 1):
    """Seeded permutation split of ``count`` systems into train / held-out."""
    perm = np.random.default_rng(seed).permutation(count)
    return perm[:n_train], perm[n_train:]


# The five workloads the hot path is measured and checked on.  Sizes follow
# the paper's n = 10 Toeplitz operating point (Section III-B/C) plus a small
# n = 3 case that the oracle finishes in seconds.
CONFIGS = {
    "toeplitz_n3_L8": dict(n=3, a=1.0, b=-0.4, tau=0.01, layers=2, seed=0,
                           cost="global", gd_steps=50, eta=0.1),
    "toeplitz_n10_L64": dict(n=10, a=1.0, b=-0.45, tau=0.01, layers=4, seed=0,
                             cost="local"),
    "toeplitz_n10_L128": dict(n=10, a=1.0, b=-0.45, tau=0.005, layers=6, seed=0,
                              cost="local"),
    "random_sym_n12": dict(n=12, seed=0),
    "heleshaw_n10_L256": dict(n=10, m=32, sigma=0.5, top_L=256, layers=6,
                              seed=0, cost="local", iters=200),
    "warmstart_n10_L64": dict(n=10, count=4096, n_train=3584, top_L=64,
                              layers=4, seed=0, cost="local"),
}
