"""The fast form's iteration replayed from HIP graphs.

One iteration (Algorithm 1's loop body with the project forms): the adjoint
gradient with complex64 states on a second stream, the 2(n+1)L^2 (local) or
2(L^2 + L) (global) Hadamard-test circuits with complex64 states on the
launch stream, both reading theta_k; the update theta_{k+1} = theta_k -
eta g_k once the gradient is there; the cost of iteration k assembled (in
float64) on the second stream beside the circuits of iteration k + 1.

Every iteration is the same fixed sequence of library launches, so it is
captured once and replayed: the per-launch host work disappears and the
cross-stream waits become graph edges.  The term buffers alternate between
consecutive iterations (the cost of one iteration reads them while the next
iteration's circuits write the other set), hence two graphs, replayed in
turn.  With `unroll` > 1, runs of that many consecutive iterations are also
captured as one graph each, so the iterations inside a run follow each
other without the gap between two graph launches.  The graphs hold no
memory set or copy nodes, only library kernels.
"""
from __future__ import annotations

import torch

from . import api


class FastGradientDescent:
    """Gradient descent on one system, theta [1, P] (float64, device) updated
    in place by every step."""

    def __init__(self, ansatz: api.AnsatzSpec, coeffs: torch.Tensor, strings: torch.Tensor, theta: torch.Tensor,
                 eta: float, kind: str = "local", b_kind: str = "plus", b: torch.Tensor | None = None,
                 unroll: int = 1):
        if unroll < 1:
            raise ValueError(f"unroll must be >= 1, got {unroll}")
        if theta.dim() != 2 or theta.shape[0] != 1 or theta.shape[1] != ansatz.P:
            raise ValueError(f"theta must be [1, {ansatz.P}], got {tuple(theta.shape)}")
        if theta.dtype != torch.float64 or not theta.is_cuda or not theta.is_contiguous():
            raise TypeError("theta must be a contiguous float64 CUDA tensor")
        self.an, self.coeffs, self.strings, self.theta, self.eta = ansatz, coeffs, strings, theta, float(eta)
        self.kind, self.b_kind, self.b = kind, b_kind, b
        dev = theta.device
        n, L, P = ansatz.n, strings.shape[0], ansatz.P
        other = (1, n, L, L) if kind == "local" else (1, L)

        def term_set():  # zeroed: the first step assembles a cost from the other set
            return (torch.zeros((1, L, L), dtype=torch.complex128, device=dev),
                    torch.zeros(other, dtype=torch.complex128, device=dev),
                    torch.zeros(1, dtype=torch.float64, device=dev),
                    torch.zeros((1, 2), dtype=torch.complex128, device=dev))

        self.bufs = [term_set(), term_set()]
        self.Ca = torch.empty(1, dtype=torch.float64, device=dev)
        self.grad = torch.empty((1, P), dtype=torch.float64, device=dev)
        self.side = torch.cuda.Stream(device=dev)  # default priority
        self.k = 0
        # eager steps on a scratch copy first: every kernel's first launch
        # (its LDS attribute) happens outside the capture
        scratch = theta.detach().clone()
        for k in range(2):
            self._step(k, scratch)
        torch.cuda.synchronize(dev)
        self.graphs = [self._capture(k, 1) for k in range(2)]
        # `unroll` consecutive iterations per graph (one per starting parity):
        # the iterations inside a graph follow each other without the gap
        # between two graph launches
        self.unroll = unroll
        self.blocks = [self._capture(k, unroll) for k in range(2)] if unroll > 1 else []
        # one replay of every graph (a graph's first launch carries one-off
        # costs), then the angles and the term buffers are put back
        saved = theta.detach().clone()
        for g in self.graphs + self.blocks:
            g.replay()
        self.theta.copy_(saved)
        for buf in self.bufs:
            for t in buf:
                t.zero_()
        torch.cuda.synchronize(dev)

    def _capture(self, k0: int, count: int) -> torch.cuda.CUDAGraph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=torch.cuda.Stream(device=self.theta.device)):
            for k in range(k0, k0 + count):
                self._step(k, self.theta)
        return g

    def _step(self, k: int, theta: torch.Tensor) -> None:
        main = torch.cuda.current_stream(theta.device)
        beta, other, _, _ = self.bufs[k & 1]
        pbeta, pother, pC, pparts = self.bufs[(k - 1) & 1]
        self.side.wait_stream(main)
        with torch.cuda.stream(self.side):
            api.vqls_grad_adjoint(self.an, theta, self.coeffs, self.strings, self.kind, "f32", b_kind=self.b_kind,
                                  b=self.b, out=(self.Ca, self.grad))
            # cost of the previous iteration, beside this iteration's circuits
            api.vqls_cost(self.coeffs, self.an.n, self.kind, pbeta, pother, out=(pC, pparts))
        api.vqls_terms(self.an, theta, self.strings, self.kind, "f32", b_kind=self.b_kind, b=self.b,
                       out=(beta, other))
        main.wait_stream(self.side)
        api.gd_step(theta, self.grad, self.eta)

    def step(self, count: int = 1) -> None:
        """`count` iterations, launched on the current stream."""
        while self.blocks and count >= self.unroll:
            self.blocks[self.k & 1].replay()
            self.k += self.unroll
            count -= self.unroll
        for _ in range(count):
            self.graphs[self.k & 1].replay()
            self.k += 1

    def last_cost(self) -> torch.Tensor:
        """Cost of the last iteration (assembled now, on the current stream);
        float64 [1]."""
        if self.k == 0:
            raise RuntimeError("no iteration has run")
        beta, other, C, parts = self.bufs[(self.k - 1) & 1]
        api.vqls_cost(self.coeffs, self.an.n, self.kind, beta, other, out=(C, parts))
        return C
