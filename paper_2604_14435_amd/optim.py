"""L-BFGS-B driver for one VQLS system (the paper's optimizer, Section III).

The optimizer itself is host-side (SciPy's L-BFGS-B on the P angles, as in
the paper); every cost and gradient it asks for is computed on the GPU by
libdvq.so:
  * fast form  ("f32"): the cost from the 2(n+1)L^2 Hadamard-test circuits
    with complex64 states (float64 accumulation), the gradient from the
    adjoint sweep with complex64 states, the two launched on separate
    streams;
  * plain form ("f64"): cost and gradient from the parameter-shift rule,
    (2P + 1) evaluations of every circuit with complex128 states;
  * adjoint forms ("f64-adjoint", "f32-adjoint"): cost and gradient from
    the adjoint sweep alone, complex128 or complex64 states (complex128: the
    same values as the plain form to rounding, the shift rule being exact
    for RY gates).
Each evaluation ends with one device-to-host copy of (cost, gradient); its
launches are replayed from a HIP graph after the first call.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


@dataclass
class Trace:
    """What one run did: costs per evaluation; per accepted iterate (L-BFGS
    iteration) the angles, the evaluations used so far and the seconds since
    the start."""
    costs: list = field(default_factory=list)
    thetas: list = field(default_factory=list)
    iter_evals: list = field(default_factory=list)
    iter_seconds: list = field(default_factory=list)
    evals: int = 0
    seconds: float = 0.0
    stop: str = ""


class Evaluator:
    """Cost and gradient of one system at one angle vector, on the GPU.

    The evaluation writes (cost, gradient) straight into one device buffer,
    copied to pinned host memory in one transfer.  With `graph` (default)
    the evaluation's launches are captured once, after a first eager call,
    and replayed: only the angles' upload, the replay and the result's
    download remain per call."""

    def __init__(self, ansatz: api.AnsatzSpec, coeffs: torch.Tensor, strings: torch.Tensor, form: str,
                 kind: str = "local", b_kind: str = "plus", b=None, graph: bool = True):
        if form not in ("f32", "f64", "f64-adjoint", "f32-adjoint"):
            raise ValueError(f"unknown form {form!r}")
        self.an, self.coeffs, self.strings, self.form = ansatz, coeffs, strings, form
        self.kind, self.b_kind, self.b = kind, b_kind, b
        dev = coeffs.device
        self.dev = dev
        L = coeffs.shape[0]
        n, P = ansatz.n, ansatz.P
        self.theta = torch.empty((1, P), dtype=torch.float64, device=dev)
        self.theta_host = torch.empty(P, dtype=torch.float64, pin_memory=True)
        self.packed = torch.empty(P + 1, dtype=torch.float64, device=dev)  # (C, grad)
        self.out_host = torch.empty(P + 1, dtype=torch.float64, pin_memory=True)
        self.C = self.packed[0:1]
        self.g = self.packed[1:].view(1, P)
        if form == "f32":
            other = (1, n, L, L) if kind == "local" else (1, L)
            self.beta = torch.empty((1, L, L), dtype=torch.complex128, device=dev)
            self.other = torch.empty(other, dtype=torch.complex128, device=dev)
            self.parts = torch.empty((1, 2), dtype=torch.complex128, device=dev)
            self.Ca = torch.empty(1, dtype=torch.float64, device=dev)
            self.side = torch.cuda.Stream(device=dev)  # default priority
        elif form == "f64":
            self.ws = api.ShiftWorkspace(ansatz, L, kind, dev)
        self.use_graph = graph
        self.graph = None

    def _launch(self) -> None:
        """The evaluation at self.theta, on the current stream."""
        main = torch.cuda.current_stream(self.dev)
        if self.form == "f32":
            self.side.wait_stream(main)
            with torch.cuda.stream(self.side):
                api.vqls_grad_adjoint(self.an, self.theta, self.coeffs, self.strings, self.kind, "f32",
                                      b_kind=self.b_kind, b=self.b, out=(self.Ca, self.g))
            api.vqls_terms(self.an, self.theta, self.strings, self.kind, "f32", b_kind=self.b_kind, b=self.b,
                           out=(self.beta, self.other))
            api.vqls_cost(self.coeffs, self.an.n, self.kind, self.beta, self.other, out=(self.C, self.parts))
            main.wait_stream(self.side)
        elif self.form == "f64":
            api.vqls_grad_shift(self.an, self.theta[0], self.coeffs, self.strings, self.kind, "f64",
                                b_kind=self.b_kind, b=self.b, workspace=self.ws, out=(self.C, self.g[0]))
        else:
            api.vqls_grad_adjoint(self.an, self.theta, self.coeffs, self.strings, self.kind, self.form[:3],
                                  b_kind=self.b_kind, b=self.b, out=(self.C, self.g))

    def __call__(self, theta: np.ndarray) -> tuple[float, np.ndarray]:
        self.theta_host.numpy()[:] = np.asarray(theta, dtype=np.float64)
        self.theta[0].copy_(self.theta_host, non_blocking=True)
        if self.graph is not None:
            self.graph.replay()
        else:
            self._launch()
            if self.use_graph:  # capture after the first (eager, validating) call
                torch.cuda.synchronize(self.dev)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=torch.cuda.Stream(device=self.dev)):
                    self._launch()
                self.graph = g
        self.out_host.copy_(self.packed)  # synchronous: waits for the evaluation
        v = self.out_host.numpy()
        return float(v[0]), v[1:].copy()


def lbfgs(evaluate, theta0: np.ndarray, max_evals: int = 2000, target: float | None = None,
          gtol: float = 1e-9, ftol: float = 1e-15, memory: int = 10, stop_when=None) -> tuple[np.ndarray, Trace]:
    """Minimise with L-BFGS-B from theta0.  Stops at convergence, after
    `max_evals` evaluations, as soon as an evaluated cost is <= target, or
    as soon as ``stop_when(theta)`` is true for an accepted iterate."""
    from scipy.optimize import minimize

    tr = Trace()
    best = [np.inf, np.asarray(theta0, dtype=np.float64).copy()]

    class _Reached(Exception):
        pass

    def fun(th):
        c, g = evaluate(th)
        tr.costs.append(c)
        tr.evals += 1
        if c < best[0]:
            best[0], best[1] = c, np.array(th, dtype=np.float64)
        if target is not None and c <= target:
            raise _Reached()
        return c, g

    t0 = time.perf_counter()

    def on_iterate(xk):
        tr.thetas.append(np.array(xk))
        tr.iter_evals.append(tr.evals)
        tr.iter_seconds.append(time.perf_counter() - t0)
        if stop_when is not None and stop_when(xk):
            raise _Reached()

    try:
        res = minimize(fun, np.asarray(theta0, dtype=np.float64), jac=True, method="L-BFGS-B",
                       callback=on_iterate,
                       options={"maxfun": max_evals, "maxiter": max_evals, "gtol": gtol, "ftol": ftol,
                                "maxcor": memory})
        tr.stop = str(res.message)
    except _Reached:
        tr.stop = "target reached"
    tr.seconds = time.perf_counter() - t0
    return best[1], tr


def lbfgs_refine(fast, precise, theta0: np.ndarray, max_evals: int = 4000, target: float | None = None,
                 gtol: float = 1e-9) -> tuple[np.ndarray, Trace]:
    """Mixed precision: L-BFGS-B on the `fast` evaluator (complex64 states)
    until it stops -- near flat regions the float32 cost no longer resolves
    the decrease of a step -- then from its best point on the `precise`
    evaluator (complex128 adjoint), within one evaluation budget.  The
    trace concatenates both phases (iterates, evaluations, seconds)."""
    th1, t1 = lbfgs(fast, theta0, max_evals=max_evals, target=target, gtol=gtol)
    if t1.stop == "target reached" or t1.evals >= max_evals:
        return th1, t1
    th2, t2 = lbfgs(precise, th1, max_evals=max_evals - t1.evals, target=target, gtol=gtol)
    tr = Trace(costs=t1.costs + t2.costs, thetas=t1.thetas + t2.thetas,
               iter_evals=t1.iter_evals + [t1.evals + e for e in t2.iter_evals],
               iter_seconds=t1.iter_seconds + [t1.seconds + x for x in t2.iter_seconds],
               evals=t1.evals + t2.evals, seconds=t1.seconds + t2.seconds,
               stop=f"float32: {t1.stop[:40]}; float64: {t2.stop[:40]}")
    return (th2 if min(t2.costs, default=np.inf) <= min(t1.costs) else th1), tr



class BatchEvaluator:
    """Cost and gradient of B rows, row r with its own system (coeffs [B, L],
    strings [B, L, 2]), from one adjoint launch per call (complex64 or
    complex128 states); host arrays in, host arrays out."""

    def __init__(self, ansatz: api.AnsatzSpec, coeffs: torch.Tensor, strings: torch.Tensor,
                 precision: str = "f64", kind: str = "local"):
        self.an, self.coeffs, self.strings = ansatz, coeffs, strings
        self.precision, self.kind = precision, kind
        dev = coeffs.device
        B, P = coeffs.shape[0], ansatz.P
        self.theta = torch.empty((B, P), dtype=torch.float64, device=dev)
        self.theta_host = torch.empty((B, P), dtype=torch.float64, pin_memory=True)
        self.packed = torch.empty((B, P + 1), dtype=torch.float64, device=dev)
        self.out_host = torch.empty((B, P + 1), dtype=torch.float64, pin_memory=True)
        self.C = torch.empty(B, dtype=torch.float64, device=dev)
        self.g = torch.empty((B, P), dtype=torch.float64, device=dev)
        self.evals = 0

    def __call__(self, theta: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
        self.theta_host.numpy()[:] = theta
        self.theta.copy_(self.theta_host, non_blocking=True)
        api.vqls_grad_adjoint(self.an, self.theta, self.coeffs, self.strings, self.kind, self.precision,
                              per_row_system=True, out=(self.C, self.g))
        self.packed[:, 0].copy_(self.C)
        self.packed[:, 1:].copy_(self.g)
        self.out_host.copy_(self.packed)  # synchronous
        self.evals += 1
        v = self.out_host.numpy()
        return v[:, 0].copy(), v[:, 1:].copy()


def lbfgs_batched(evaluate, theta0: np.ndarray, iters: int = 300, memory: int = 10, c1: float = 1e-4,
                  max_backtracks: int = 20) -> tuple[np.ndarray, np.ndarray]:
    """B independent L-BFGS minimisations advanced together (host-side, as
    the paper's optimizer), each row with its own curvature pairs and its own
    Armijo backtracking step; every call of ``evaluate(theta [B, P]) ->
    (C [B], grad [B, P])`` evaluates all rows at once, rows not searching a
    step being evaluated at their current point.  A row whose direction is
    not a descent direction restarts from the gradient with an empty memory;
    pairs with s.y <= 0 are not stored.  Returns (theta [B, P], C [B])."""
    x = np.array(theta0, dtype=np.float64, copy=True)
    B, P = x.shape
    f, g = evaluate(x)
    S = np.zeros((memory, B, P))
    Y = np.zeros((memory, B, P))
    rho = np.zeros((memory, B))
    count = np.zeros(B, dtype=np.int64)  # stored pairs per row (ring buffer, newest at count-1)
    for _ in range(iters):
        # two-loop recursion, every row with its own pairs (empty slots have rho = 0)
        q = -g.copy()
        alpha = np.zeros((memory, B))
        for back in range(memory):
            slot = (count - 1 - back) % memory
            valid = back < np.minimum(count, memory)
            s_k, y_k, r_k = S[slot, np.arange(B)], Y[slot, np.arange(B)], rho[slot, np.arange(B)] * valid
            alpha[back] = r_k * np.einsum("bp,bp->b", s_k, q)
            q -= alpha[back][:, None] * y_k
        last = (count - 1) % memory
        s_l, y_l = S[last, np.arange(B)], Y[last, np.arange(B)]
        yy = np.einsum("bp,bp->b", y_l, y_l)
        gamma = np.where(count > 0, np.einsum("bp,bp->b", s_l, y_l) / np.where(yy > 0, yy, 1.0), 1.0)
        q *= gamma[:, None]
        for back in reversed(range(memory)):
            slot = (count - 1 - back) % memory
            valid = back < np.minimum(count, memory)
            s_k, y_k, r_k = S[slot, np.arange(B)], Y[slot, np.arange(B)], rho[slot, np.arange(B)] * valid
            beta = r_k * np.einsum("bp,bp->b", y_k, q)
            q += (alpha[back] - beta)[:, None] * s_k
        d = q
        gd = np.einsum("bp,bp->b", g, d)
        bad = gd >= 0
        if bad.any():  # restart those rows from steepest descent
            d[bad] = -g[bad]
            gd[bad] = -np.einsum("bp,bp->b", g[bad], g[bad])
            count[bad] = 0
        gnorm = np.sqrt(np.einsum("bp,bp->b", g, g))
        t = np.where(count > 0, 1.0, np.minimum(1.0, 1.0 / np.maximum(gnorm, 1e-300)))
        pending = gd < 0
        x_new, f_new, g_new = x.copy(), f.copy(), g.copy()
        for _ls in range(max_backtracks):
            if not pending.any():
                break
            trial = np.where(pending[:, None], x + t[:, None] * d, x)
            ft, gt = evaluate(trial)
            ok = pending & (ft <= f + c1 * t * gd)
            x_new[ok], f_new[ok], g_new[ok] = trial[ok], ft[ok], gt[ok]
            pending &= ~ok
            t = np.where(pending, 0.5 * t, t)
        accepted = ~pending & (gd < 0)
        s = x_new - x
        y = g_new - g
        sy = np.einsum("bp,bp->b", s, y)
        store = accepted & (sy > 1e-300)
        slot = count % memory
        rows = np.nonzero(store)[0]
        S[slot[rows], rows] = s[rows]
        Y[slot[rows], rows] = y[rows]
        rho[slot[rows], rows] = 1.0 / sy[rows]
        count[rows] += 1
        count[pending] = 0  # no acceptable step: restart that row's memory
        x, f, g = x_new, f_new, g_new
    return x, f
