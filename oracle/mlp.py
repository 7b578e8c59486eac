"""FP64 reference of the warm-start MLP -- oracle (test infrastructure only).

The paper has no learned component; this network is a project form of the
hot path: it maps a system descriptor to initial ansatz angles.  Shape
d_in -> 256 -> 256 -> P with ReLU hidden activations:
    h1 = relu(X W1^T + b1),  h2 = relu(h1 W2^T + b2),  y = h2 W3^T + b3.
The GPU path rounds every GEMM operand (weights, activations, output
gradients) to bfloat16 and accumulates in FP32; the reference applies the
same rounding at the same points (``bf16=True``) and computes in FP64.

Loss (wrap-safe for angles): mean over batch and outputs of 1 - cos(y - t).
Optimizer: Adam with decoupled weight decay (AdamW), FP32 master weights on
the GPU, FP64 here.

Pins: backward == central finite differences of the forward (bf16=False),
Adam step against its closed form after one step (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

LAYERS = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    Goes through float32 first (the GPU operands are FP32 values)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(d_in: int, hidden: int, d_out: int, seed: int = 0) -> dict:
    """He-uniform weights, zero biases (FP64 copies of FP32 values)."""
    rng = np.random.default_rng(seed)

    def w(o, i):
        lim = np.sqrt(6.0 / i)
        return rng.uniform(-lim, lim, size=(o, i)).astype(np.float32).astype(np.float64)

    return dict(W1=w(hidden, d_in), b1=np.zeros(hidden), W2=w(hidden, hidden), b2=np.zeros(hidden),
                W3=w(d_out, hidden), b3=np.zeros(d_out))


def _q(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(p: dict, X: np.ndarray, bf16: bool = True):
    """Returns (y, cache)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = _q(X, bf16) @ _q(p["W1"], bf16).T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _q(h1, bf16) @ _q(p["W2"], bf16).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = _q(h2, bf16) @ _q(p["W3"], bf16).T + p["b3"]
    return y, dict(X=X, h1=h1, h2=h2)


def loss_and_grad_output(y: np.ndarray, t: np.ndarray):
    """l = mean(1 - cos(y - t)); dl/dy = sin(y - t) / y.size."""
    d = y - t
    return float(np.mean(1.0 - np.cos(d))), np.sin(d) / d.size


def backward(p: dict, cache: dict, dy: np.ndarray, bf16: bool = True) -> dict:
    X, h1, h2 = cache["X"], cache["h1"], cache["h2"]
    g = {}
    dyq = _q(dy, bf16)
    g["W3"] = dyq.T @ _q(h2, bf16)
    g["b3"] = dy.sum(axis=0)
    dh2 = dyq @ _q(p["W3"], bf16)
    dz2 = dh2 * (h2 > 0)
    dz2q = _q(dz2, bf16)
    g["W2"] = dz2q.T @ _q(h1, bf16)
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2q @ _q(p["W2"], bf16)
    dz1 = dh1 * (h1 > 0)
    dz1q = _q(dz1, bf16)
    g["W1"] = dz1q.T @ _q(X, bf16)
    g["b1"] = dz1.sum(axis=0)
    return g


def adamw_step(p: dict, g: dict, m: dict, v: dict, t: int, lr=1e-3, beta1=0.9, beta2=0.999,
               eps=1e-8, weight_decay=0.0):
    """One AdamW step (t counts from 1); updates p, m, v in place."""
    for k in LAYERS:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * (mh / (np.sqrt(vh) + eps) + weight_decay * p[k])
    return p, m, v
