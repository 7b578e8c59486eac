"""Learned warm start for the VQLS angles (a project form around the method).

Pipeline, every arithmetic step in libdvq.so kernels (Python only orders the
calls and moves tensors):
  1. decompose each system of a family on the GPU (top-L Pauli terms);
  2. generate training angles with the solver itself: gradient descent with
     the adjoint gradient, all systems batched in one launch per iteration,
     every system started from one common angle vector (the solution of a
     reference system), so the optimised angles vary smoothly over the family;
  3. train the bfloat16 MLP (descriptor -> angles) with the wrap-safe loss
     mean(1 - cos(pred - target)) and AdamW, one fused kernel pair per
     minibatch (inputs standardised on the device);
  4. predict initial angles for new systems; random initialisation remains
     the reference and the fallback (a prediction whose cost is not finite or
     is worse than the random start's is replaced by the random start).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from . import api


def decompose_batches(batches, top_L: int) -> tuple[torch.Tensor, torch.Tensor, np.ndarray]:
    """Top-L terms of every matrix of an iterable of device batches [b, N, N]
    (one batched call per batch): coeffs [S, L] complex128, strings
    [S, L, 2] int32, relative Frobenius errors [S]."""
    cs, ss, fe = [], [], []
    ws = None
    for A in batches:
        n = A.shape[1].bit_length() - 1
        need = L.load().dvq_decompose_batch_workspace_bytes(n, A.shape[0])
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=A.device)
        c, s, f = api.pauli_decompose_batch(A, top_L, workspace=ws)
        cs.append(c)
        ss.append(s)
        fe.append(f)
    return torch.cat(cs), torch.cat(ss), np.concatenate(fe)


def decompose_family(matrices, top_L: int, device, chunk: int = 256
                     ) -> tuple[torch.Tensor, torch.Tensor, np.ndarray]:
    """Top-L terms of each host matrix of an iterable, `chunk` per batched call."""
    import itertools

    it = iter(matrices)

    def batches():
        while True:
            part = list(itertools.islice(it, chunk))
            if not part:
                return
            yield torch.from_numpy(np.stack(part)).to(device)

    return decompose_batches(batches(), top_L)


def toeplitz_batches(ab: np.ndarray, n: int, device, chunk: int = 256):
    """The tridiagonal Toeplitz matrices of the (a, b) pairs (diagonal a,
    both off-diagonals b: the same matrices as workloads.toeplitz(n, a, b)),
    built in device memory `chunk` at a time; yields [b, N, N] float64."""
    N = 1 << n
    idx = torch.arange(N, device=device)
    for s0 in range(0, len(ab), chunk):
        part = torch.as_tensor(np.ascontiguousarray(ab[s0:s0 + chunk]), dtype=torch.float64, device=device)
        A = torch.zeros((part.shape[0], N, N), dtype=torch.float64, device=device)
        A[:, idx, idx] = part[:, 0:1]
        A[:, idx[:-1], idx[:-1] + 1] = part[:, 1:2]
        A[:, idx[:-1] + 1, idx[:-1]] = part[:, 1:2]
        yield A


def solve(ansatz: api.AnsatzSpec, coeffs, strings, theta0: torch.Tensor, iters: int, lr: float,
          kind: str = "local", precision: str = "f32", per_row_system: bool = True,
          record: bool = True):
    """Gradient descent with the adjoint gradient for B rows at once.

    Returns (theta [B, P], costs [iters + 1, B] or None); costs[t] is the cost
    at the iterate after t steps."""
    theta = theta0.clone().contiguous()
    B = theta.shape[0]
    C = torch.empty(B, dtype=torch.float64, device=theta.device)
    g = torch.empty((B, ansatz.P), dtype=torch.float64, device=theta.device)
    hist = torch.empty((iters + 1, B), dtype=torch.float64, device=theta.device) if record else None
    for t in range(iters):
        api.vqls_grad_adjoint(ansatz, theta, coeffs, strings, kind, precision,
                              per_row_system=per_row_system, out=(C, g))
        if record:
            hist[t].copy_(C)
        api.gd_step(theta, g, lr)
    if record:
        api.vqls_grad_adjoint(ansatz, theta, coeffs, strings, kind, precision,
                              per_row_system=per_row_system, out=(C, g))
        hist[iters].copy_(C)
    return theta, hist


def iterations_to(costs: torch.Tensor, threshold: torch.Tensor) -> torch.Tensor:
    """First iteration index t with costs[t, b] <= threshold[b]; -1 if never."""
    hit = costs <= threshold.unsqueeze(0)
    idx = torch.where(hit.any(0), hit.float().argmax(0), torch.full_like(hit[0], -1, dtype=torch.long))
    return idx.long()


@dataclass
class MLPConfig:
    hidden: int = 256
    epochs: int = 300
    batch: int = 256
    lr: float = 1e-3
    weight_decay: float = 0.0
    seed: int = 0


class WarmStartMLP:
    """d_in -> hidden -> hidden -> P network on the bfloat16 matrix cores.

    Training and inference run the fused kernels (dvq_mlp_train_step: one
    minibatch step in three launches; dvq_mlp_predict): the input
    standardisation statistics are computed by the library
    (dvq_feature_stats) and applied inside the kernels; Python only draws
    the epoch's row permutation (host generator) and orders the calls."""

    def __init__(self, d_in: int, d_out: int, cfg: MLPConfig = MLPConfig(), device="cuda:0", out_bias=None):
        """`out_bias` (length d_out) initialises the output layer's bias: with
        the solution of a reference system there, training fits each
        system's offset from that solution rather than its absolute angles."""
        if d_in > 32 or d_out > 128 or cfg.hidden not in (64, 128, 256):
            raise ValueError("the fused MLP kernels take d_in <= 32, d_out <= 128, hidden 64/128/256")
        self.cfg = cfg
        self.device = torch.device(device)
        self.shape = api.mlp_shape(d_in, cfg.hidden, d_out)
        self.params = self.init_params(d_in, cfg.hidden, d_out, cfg.seed, out_bias).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.stats = None  # (mean, 1/std) of the training inputs, device float32

    @staticmethod
    def init_params(d_in: int, hidden: int, d_out: int, seed: int, out_bias=None) -> torch.Tensor:
        """He-uniform weights, zero biases (b3 = out_bias when given), packed
        W1, b1, W2, b2, W3, b3."""
        rng = np.random.default_rng(seed)

        def w(o, i):
            lim = math.sqrt(6.0 / i)
            return rng.uniform(-lim, lim, size=(o, i)).astype(np.float32).ravel()

        z = lambda k: np.zeros(k, dtype=np.float32)
        b3 = z(d_out) if out_bias is None else np.asarray(out_bias, dtype=np.float32).reshape(d_out)
        flat = np.concatenate([w(hidden, d_in), z(hidden), w(hidden, hidden), z(hidden),
                               w(d_out, hidden), b3])
        return torch.from_numpy(flat)

    def fit(self, X, T, epochs: int | None = None):
        """Train on descriptors X [S, d_in] and angles T [S, P]; returns the
        per-epoch mean loss (float64 numpy)."""
        cfg = self.cfg
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        T = torch.as_tensor(T, dtype=torch.float32, device=self.device).contiguous()
        self.stats = api.feature_stats(X)
        S = X.shape[0]
        bs = min(cfg.batch, S)
        steps = S // bs
        n_ep = epochs if epochs is not None else cfg.epochs
        gen = torch.Generator().manual_seed(cfg.seed)
        ws = api.TrainWorkspace(self.shape, bs, self.device)
        losses = torch.empty(n_ep * steps, dtype=torch.float64, device=self.device)
        # every epoch's row permutation, drawn on the host and uploaded once
        perms = torch.stack([torch.randperm(S, generator=gen) for _ in range(n_ep)]).to(torch.int32)
        perms = perms.to(self.device)
        for e in range(n_ep):
            for j in range(steps):
                self.t += 1
                k = e * steps + j
                api.mlp_train_step(self.shape, self.params, self.m, self.v, self.t, X, T,
                                   rows=perms[e, j * bs:(j + 1) * bs], stats=self.stats, lr=cfg.lr,
                                   weight_decay=cfg.weight_decay, workspace=ws, loss=losses[k:k + 1])
        return losses.cpu().numpy().reshape(n_ep, steps).mean(axis=1)

    def predict(self, X) -> torch.Tensor:
        """Initial angles [S, P] as float64."""
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        return api.mlp_predict(self.shape, self.params, X, stats=self.stats).double()


def choose_start(ansatz, coeffs, strings, theta_pred, theta_rand, kind="local", precision="f32"):
    """Fallback rule: keep the predicted start where its cost is finite and not
    worse than the random start's, else use the random start.  Returns
    (theta0 [S, P], used_prediction bool [S])."""
    Cp, _ = api.vqls_grad_adjoint(ansatz, theta_pred, coeffs, strings, kind, precision, per_row_system=True)
    Cr, _ = api.vqls_grad_adjoint(ansatz, theta_rand, coeffs, strings, kind, precision, per_row_system=True)
    use = torch.isfinite(Cp) & (Cp <= Cr)
    return torch.where(use.unsqueeze(1), theta_pred, theta_rand), use


def race_starts(ansatz: api.AnsatzSpec, coeffs: torch.Tensor, strings: torch.Tensor, theta_pred: np.ndarray,
                theta_ref: np.ndarray, iters: int = 8, kind: str = "local", precision: str = "f32"):
    """Start selection by a short race: for every system (coeffs [S, L],
    strings [S, L, 2]) both starts, the prediction and the reference (e.g.
    V|0> = b), take `iters` L-BFGS iterations together (one batched adjoint
    launch per evaluation of all 2S rows); each system keeps the run that
    reached the lower cost.  A start whose cost is lower is not always the
    one that converges sooner, which the race settles at a small fixed cost.
    Returns (theta [S, P], the winning runs' iterates; used_prediction [S]
    bool; C [S], their costs; evaluations of the batched race)."""
    from .optim import BatchEvaluator, lbfgs_batched

    S = coeffs.shape[0]
    both = np.concatenate([np.asarray(theta_pred, dtype=np.float64).reshape(S, -1),
                           np.broadcast_to(np.asarray(theta_ref, dtype=np.float64), (S, ansatz.P))])
    ev = BatchEvaluator(ansatz, torch.cat([coeffs, coeffs]).contiguous(), torch.cat([strings, strings]).contiguous(),
                        precision, kind)
    th, C = lbfgs_batched(ev, both, iters=iters)
    use = np.isfinite(C[:S]) & (C[:S] <= C[S:])
    return np.where(use[:, None], th[:S], th[S:]), use, np.where(use, C[:S], C[S:]), ev.evals


def continuation_targets(ansatz: api.AnsatzSpec, ab: np.ndarray, coeffs: torch.Tensor, strings: torch.Tensor,
                         theta_centre: np.ndarray, centre, bins: int = 16, iters: int = 100,
                         precision: str = "f64", kind: str = "local") -> tuple[np.ndarray, np.ndarray]:
    """Training angles for a family by continuation in the off-diagonal b:
    the family is cut into `bins` bins of b; the bin holding the centre
    system starts from its solution, and every further bin, taken outward
    from there, starts each system from the solution of the nearest
    already-solved system in (a, b).  Each bin is solved by one batched
    L-BFGS run (complex128 adjoint).  Neighbouring systems thus start close
    to each other's solutions and stay on one branch of the solution set,
    which is what a network can interpolate.  Returns (theta [S, P],
    final cost [S])."""
    from .optim import BatchEvaluator, lbfgs_batched

    S = len(ab)
    edges = np.linspace(ab[:, 1].min(), ab[:, 1].max() + 1e-12, bins + 1)
    which = np.clip(np.searchsorted(edges, ab[:, 1], side="right") - 1, 0, bins - 1)
    c_bin = int(np.clip(np.searchsorted(edges, centre[1], side="right") - 1, 0, bins - 1))
    order = [c_bin] + [b for d in range(1, bins) for b in (c_bin - d, c_bin + d) if 0 <= b < bins]
    theta = np.zeros((S, ansatz.P))
    cost = np.full(S, np.inf)
    solved = np.zeros(S, dtype=bool)
    for b in order:
        idx = np.nonzero(which == b)[0]
        if len(idx) == 0:
            continue
        if not solved.any():
            start = np.tile(theta_centre, (len(idx), 1))
        else:
            done = np.nonzero(solved)[0]
            d2 = ((ab[idx, None, :] - ab[None, done, :]) ** 2).sum(-1)
            start = theta[done[np.argmin(d2, axis=1)]]
        sel = torch.from_numpy(idx).to(coeffs.device)
        ev = BatchEvaluator(ansatz, coeffs[sel].contiguous(), strings[sel].contiguous(), precision, kind)
        th, f = lbfgs_batched(ev, start, iters=iters)
        theta[idx], cost[idx] = th, f
        solved[idx] = True
    return theta, cost
