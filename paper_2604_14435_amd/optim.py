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
          gtol: float = 1e-9, ftol: float = 1e-15, memory: int = 10) -> tuple[np.ndarray, Trace]:
    """Minimise with L-BFGS-B from theta0.  Stops at convergence, after
    `max_evals` evaluations, or as soon as an evaluated cost is <= target."""
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

