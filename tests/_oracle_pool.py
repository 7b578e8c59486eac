"""Run the oracle's Hadamard-test circuits of one whole cost evaluation in a
process pool (test infrastructure; imports only the oracle and numpy).

The pool uses the "spawn" start method, so its workers are fresh
interpreters that never touch the GPU, even when the calling process has.

Circuit order of one evaluation (local cost): circuit c = 2u + part, part 1
is the imaginary-part circuit (S^dagger before the final H); term
u = j L^2 + l L + m, with j = 0 the beta_lm term and j >= 1 the delta term
of qubit j - 1 (Section II-B after Eq. (4): 2(n+1)L^2 circuits).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_S = {}


def _init(n, layers, ent, xs, zs, theta):
    _S.update(n=n, layers=layers, ent=ent, xs=np.asarray(xs), zs=np.asarray(zs),
              th=np.asarray(theta, dtype=np.float64), L=len(xs))


def _circuit(c: int) -> float:
    from oracle import circuit as qc

    n, layers, ent, xs, zs, th, L = (_S[k] for k in ("n", "layers", "ent", "xs", "zs", "th", "L"))
    part, u = c & 1, c >> 1
    jj, lm = divmod(u, L * L)
    l, m = divmod(lm, L)
    sl, sm = (int(xs[l]), int(zs[l])), (int(xs[m]), int(zs[m]))
    if jj == 0:
        return qc.beta_circuit(th, n, layers, ent, sl, sm, bool(part))
    return qc.delta_circuit(th, n, layers, ent, sl, sm, jj - 1, bool(part))


def _range(bounds):
    return [_circuit(c) for c in range(*bounds)]


def workers() -> int:
    """At most 16 processes (the CPU share of one GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def local_terms(n, layers, ent, xs, zs, theta, procs=None):
    """Every term of one local-cost evaluation through the oracle's circuits:
    (beta[L, L], delta[n, L, L]) complex128."""
    L = len(xs)
    total = 2 * (n + 1) * L * L
    procs = procs or workers()
    step = -(-total // (8 * procs))
    chunks = [(c0, min(c0 + step, total)) for c0 in range(0, total, step)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs, initializer=_init, initargs=(n, layers, ent, list(xs), list(zs), list(theta))) as pool:
        vals = np.array([v for part in pool.map(_range, chunks) for v in part])
    terms = (vals[0::2] + 1j * vals[1::2]).reshape(n + 1, L, L)
    return terms[0], terms[1:]
