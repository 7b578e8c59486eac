"""Torch-facing wrappers of the C ABI: argument marshalling only.

Every function takes CUDA (HIP) tensors, passes their device pointers and
the current stream to libdvq.so, and returns tensors allocated by torch.  No
arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

ENTANGLERS = {"cz": L.DVQ_ENT_CZ_LADDER, "cnot": L.DVQ_ENT_CNOT_LADDER}
KINDS = {"global": L.DVQ_COST_GLOBAL, "local": L.DVQ_COST_LOCAL}
PRECISIONS = {"f64": L.DVQ_F64, "f32": L.DVQ_F32}
EXECS = {"literal": L.DVQ_EXEC_LITERAL, "generic": L.DVQ_EXEC_GENERIC, "shared": L.DVQ_EXEC_SHARED}


@dataclass(frozen=True)
class AnsatzSpec:
    """V(theta): `layers` layers of RY on each of `n` qubits + a ladder."""
    n: int
    layers: int
    entangler: str = "cz"

    @property
    def P(self) -> int:
        return self.n * self.layers

    def c(self) -> L.Ansatz:
        return L.Ansatz(self.n, self.layers, ENTANGLERS[self.entangler])


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(t: torch.Tensor | None = None):
    dev = t.device if t is not None else None
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _cuda(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def _shape(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    """The kernels index inputs by the sizes they are given: check them here."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _out(t, shape, dtype, name: str) -> torch.Tensor:
    """A caller-supplied output: CUDA, contiguous, of the exact dtype and shape
    the kernels write (they cannot check a pointer's extent)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return _shape(t, shape, name)


def _square(A: torch.Tensor) -> torch.Tensor:
    """A [N, N] with N a power of two."""
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.shape[0] < 2 or A.shape[0] & (A.shape[0] - 1):
        raise ValueError(f"A must be [N, N] with N = 2^n >= 2, got {tuple(A.shape)}")
    return A


def _b_args(b_kind: str, b):
    if b_kind == "plus":
        return L.DVQ_B_PLUS, None
    return L.DVQ_B_VECTOR, _cuda(b, torch.float64, "b")


# -------------------------------------------------------------- decomposition

def decompose_workspace(n: int, device) -> torch.Tensor:
    """Scratch buffer for pauli_decompose(_dense) at n qubits."""
    return torch.empty(max(1, L.load().dvq_decompose_workspace_bytes(n)), dtype=torch.uint8, device=device)


def pauli_decompose_dense(A: torch.Tensor, out: torch.Tensor | None = None,
                          workspace: torch.Tensor | None = None) -> torch.Tensor:
    """All 4^n coefficients, complex128 [N, N] indexed [x, z]."""
    A = _square(_cuda(A, torch.float64, "A"))
    N = A.shape[0]
    n = N.bit_length() - 1
    ws = decompose_workspace(n, A.device) if workspace is None else workspace
    if out is None:
        out = torch.empty((N, N), dtype=torch.complex128, device=A.device)
    else:
        _out(out, (N, N), torch.complex128, "out")
    L.call("dvq_pauli_decompose_dense", _p(A), n, _p(out), _p(ws), ws.numel(), _stream(A))
    return out


def pauli_decompose(A: torch.Tensor, tau: float | None = None, top_L: int | None = None,
                    capacity: int = 65536):
    """Kept terms in ranking order: (coeffs complex128 [L], strings int32 [L, 2] = (x, z),
    relative Frobenius error)."""
    A = _square(_cuda(A, torch.float64, "A"))
    N = A.shape[0]
    n = N.bit_length() - 1
    lib = L.load()
    ws = torch.empty(lib.dvq_decompose_workspace_bytes(n), dtype=torch.uint8, device=A.device)
    coeffs = torch.empty(capacity, dtype=torch.complex128, device=A.device)
    strings = torch.empty((capacity, 2), dtype=torch.int32, device=A.device)
    lout = ctypes.c_int64(0)
    ferr = ctypes.c_double(0.0)
    L.call("dvq_pauli_decompose", _p(A), n, float(tau if tau is not None else 0.0),
           int(top_L if top_L is not None else 0), _p(coeffs), _p(strings), capacity,
           ctypes.byref(lout), ctypes.byref(ferr), _p(ws), ws.numel(), _stream(A))
    k = lout.value
    return coeffs[:k].clone(), strings[:k].clone(), ferr.value


def pauli_decompose_batch(A: torch.Tensor, top_L: int, workspace: torch.Tensor | None = None):
    """Top-L terms of each of B matrices A [B, N, N]: (coeffs complex128 [B, L],
    strings int32 [B, L, 2], relative Frobenius errors float64 numpy [B])."""
    A = _cuda(A, torch.float64, "A")
    if A.dim() != 3:
        raise ValueError(f"A must be [B, N, N], got {tuple(A.shape)}")
    _square(A[0])
    B, N = A.shape[0], A.shape[1]
    n = N.bit_length() - 1
    need = L.load().dvq_decompose_batch_workspace_bytes(n, B)
    ws = workspace if workspace is not None and workspace.numel() >= need else \
        torch.empty(need, dtype=torch.uint8, device=A.device)
    coeffs = torch.empty((B, top_L), dtype=torch.complex128, device=A.device)
    strings = torch.empty((B, top_L, 2), dtype=torch.int32, device=A.device)
    ferr = (ctypes.c_double * B)()
    L.call("dvq_pauli_decompose_batch", _p(A), n, B, int(top_L), _p(coeffs), _p(strings), ferr, _p(ws),
           ws.numel(), _stream(A))
    return coeffs, strings, np.array(ferr[:], dtype=np.float64)


def pauli_sum_dense(coeffs: torch.Tensor, strings: torch.Tensor, n: int) -> torch.Tensor:
    """sum_l c_l P_l as a dense complex128 [2^n, 2^n] matrix."""
    coeffs = _cuda(coeffs, torch.complex128, "coeffs")
    strings = _cuda(strings, torch.int32, "strings")
    _shape(strings, (coeffs.shape[0], 2), "strings")
    N = 1 << n
    out = torch.empty((N, N), dtype=torch.complex128, device=coeffs.device)
    L.call("dvq_pauli_sum_dense", _p(coeffs), _p(strings), coeffs.shape[0], n, _p(out), _stream(coeffs))
    return out


# -------------------------------------------------------------- circuits / cost

def circuit_count(n: int, L_: int, kind: str) -> int:
    return int(L.load().dvq_circuit_count(n, L_, KINDS[kind]))


def vqls_terms(ansatz: AnsatzSpec, theta: torch.Tensor, strings: torch.Tensor, kind: str = "local",
               precision: str = "f64", b_kind: str = "plus", b: torch.Tensor | None = None,
               exec_: str = "literal", out=None):
    """(beta [B, L, L], other) complex128; other = delta [B, n, L, L] or gamma [B, L]."""
    theta = _cuda(theta, torch.float64, "theta")
    if theta.dim() == 1:
        theta = theta.unsqueeze(0)
    strings = _cuda(strings, torch.int32, "strings")
    B, Lt, n = theta.shape[0], strings.shape[0], ansatz.n
    _shape(theta, (B, ansatz.P), "theta")
    _shape(strings, (Lt, 2), "strings")
    oshape = (B, n, Lt, Lt) if kind == "local" else (B, Lt)
    if out is None:
        beta = torch.empty((B, Lt, Lt), dtype=torch.complex128, device=theta.device)
        other = torch.empty(oshape, dtype=torch.complex128, device=theta.device)
    else:
        beta = _out(out[0], (B, Lt, Lt), torch.complex128, "beta")
        other = _out(out[1], oshape, torch.complex128, "other")
    bk, bt = _b_args(b_kind, b)
    if bt is not None:
        _shape(bt, (1 << n,), "b")
    a = ansatz.c()
    L.call("dvq_vqls_terms", ctypes.byref(a), _p(theta), B, PRECISIONS[precision], _p(strings), Lt,
           bk, _p(bt), KINDS[kind], EXECS[exec_], _p(beta), _p(other), _stream(theta))
    return beta, other


def vqls_terms_rhs(ansatz: AnsatzSpec, theta: torch.Tensor, strings: torch.Tensor, b: torch.Tensor,
                   kind: str = "local", precision: str = "f64", exec_: str = "literal", out=None):
    """Several right-hand sides b [R, 2^n] (real unit vectors) at the same
    angles: (beta [B, L, L] once, other [R, B, ...]) complex128, block r as
    vqls_terms with b_kind="vector", b=b[r]."""
    theta = _cuda(theta, torch.float64, "theta")
    if theta.dim() == 1:
        theta = theta.unsqueeze(0)
    strings = _cuda(strings, torch.int32, "strings")
    b = _cuda(b, torch.float64, "b")
    if b.dim() != 2 or b.shape[1] != 1 << ansatz.n:
        raise ValueError(f"b must be [R, {1 << ansatz.n}], got {tuple(b.shape)}")
    B, Lt, n, R = theta.shape[0], strings.shape[0], ansatz.n, b.shape[0]
    _shape(theta, (B, ansatz.P), "theta")
    _shape(strings, (Lt, 2), "strings")
    oshape = (R, B, n, Lt, Lt) if kind == "local" else (R, B, Lt)
    if out is None:
        beta = torch.empty((B, Lt, Lt), dtype=torch.complex128, device=theta.device)
        other = torch.empty(oshape, dtype=torch.complex128, device=theta.device)
    else:
        beta = _out(out[0], (B, Lt, Lt), torch.complex128, "beta")
        other = _out(out[1], oshape, torch.complex128, "other")
    a = ansatz.c()
    L.call("dvq_vqls_terms_rhs", ctypes.byref(a), _p(theta), B, PRECISIONS[precision], _p(strings), Lt, R,
           _p(b), KINDS[kind], EXECS[exec_], _p(beta), _p(other), _stream(theta))
    return beta, other


def vqls_cost(coeffs: torch.Tensor, n: int, kind: str, beta: torch.Tensor, other: torch.Tensor,
              out=None):
    """(C [B] float64, parts [B, 2] complex128 = (E or G, Psi))."""
    coeffs = _cuda(coeffs, torch.complex128, "coeffs")
    beta = _cuda(beta, torch.complex128, "beta")
    other = _cuda(other, torch.complex128, "other")
    B, Lt = beta.shape[0], coeffs.shape[0]
    _shape(coeffs, (Lt,), "coeffs")
    _shape(beta, (B, Lt, Lt), "beta")
    _shape(other, (B, n, Lt, Lt) if kind == "local" else (B, Lt), "other")
    if out is None:
        C = torch.empty(B, dtype=torch.float64, device=beta.device)
        parts = torch.empty((B, 2), dtype=torch.complex128, device=beta.device)
    else:
        C = _out(out[0], (B,), torch.float64, "C")
        parts = _out(out[1], (B, 2), torch.complex128, "parts")
    L.call("dvq_vqls_cost", _p(coeffs), coeffs.shape[0], n, KINDS[kind], _p(beta), _p(other), B,
           _p(C), _p(parts), _stream(beta))
    return C, parts


class ShiftWorkspace:
    """Scratch memory of the parameter-shift gradient, allocated once."""

    def __init__(self, ansatz: AnsatzSpec, L_: int, kind: str, device):
        a = ansatz.c()
        nbytes = L.load().dvq_grad_shift_workspace_bytes(ctypes.byref(a), L_, KINDS[kind])
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)


def vqls_grad_shift(ansatz: AnsatzSpec, theta: torch.Tensor, coeffs: torch.Tensor,
                    strings: torch.Tensor, kind: str = "local", precision: str = "f64",
                    b_kind: str = "plus", b=None, workspace: ShiftWorkspace | None = None, out=None):
    """Plain path: (C [1], grad [P]) by the parameter-shift rule."""
    theta = _cuda(theta, torch.float64, "theta").reshape(-1)
    coeffs = _cuda(coeffs, torch.complex128, "coeffs")
    strings = _cuda(strings, torch.int32, "strings")
    Lt = strings.shape[0]
    _shape(theta, (ansatz.P,), "theta")
    _shape(coeffs, (Lt,), "coeffs")
    _shape(strings, (Lt, 2), "strings")
    if workspace is None:
        workspace = ShiftWorkspace(ansatz, Lt, kind, theta.device)
    if out is None:
        C = torch.empty(1, dtype=torch.float64, device=theta.device)
        grad = torch.empty(ansatz.P, dtype=torch.float64, device=theta.device)
    else:
        C = _out(out[0], (1,), torch.float64, "C")
        grad = _out(out[1], (ansatz.P,), torch.float64, "grad")
    bk, bt = _b_args(b_kind, b)
    a = ansatz.c()
    L.call("dvq_vqls_grad_shift", ctypes.byref(a), _p(theta), PRECISIONS[precision], _p(coeffs),
           _p(strings), strings.shape[0], bk, _p(bt), KINDS[kind], _p(C), _p(grad),
           _p(workspace.buf), workspace.buf.numel(), _stream(theta))
    return C, grad


def vqls_grad_shift_noalloc(ansatz: AnsatzSpec, theta: torch.Tensor, coeffs: torch.Tensor,
                            strings: torch.Tensor, kind: str = "local", precision: str = "f64",
                            b_kind: str = "plus", b=None, out=None):
    """Plain path without a workspace: (C [1], grad [P]) by the parameter-shift
    rule, the library's per-GPU device scratch holding the intermediate terms."""
    theta = _cuda(theta, torch.float64, "theta").reshape(-1)
    coeffs = _cuda(coeffs, torch.complex128, "coeffs")
    strings = _cuda(strings, torch.int32, "strings")
    Lt = strings.shape[0]
    _shape(theta, (ansatz.P,), "theta")
    _shape(coeffs, (Lt,), "coeffs")
    _shape(strings, (Lt, 2), "strings")
    if out is None:
        C = torch.empty(1, dtype=torch.float64, device=theta.device)
        grad = torch.empty(ansatz.P, dtype=torch.float64, device=theta.device)
    else:
        C = _out(out[0], (1,), torch.float64, "C")
        grad = _out(out[1], (ansatz.P,), torch.float64, "grad")
    bk, bt = _b_args(b_kind, b)
    a = ansatz.c()
    L.call("dvq_vqls_grad_shift_noalloc", ctypes.byref(a), _p(theta), PRECISIONS[precision], _p(coeffs),
           _p(strings), strings.shape[0], bk, _p(bt), KINDS[kind], _p(C), _p(grad), _stream(theta))
    return C, grad


def vqls_grad_adjoint(ansatz: AnsatzSpec, theta: torch.Tensor, coeffs: torch.Tensor,
                      strings: torch.Tensor, kind: str = "local", precision: str = "f32",
                      b_kind: str = "plus", b=None, per_row_system: bool = False, out=None):
    """Fast path: (C [B], grad [B, P]) by the adjoint sweep."""
    theta = _cuda(theta, torch.float64, "theta")
    if theta.dim() == 1:
        theta = theta.unsqueeze(0)
    coeffs = _cuda(coeffs, torch.complex128, "coeffs")
    strings = _cuda(strings, torch.int32, "strings")
    B = theta.shape[0]
    Lt = strings.shape[-2]
    _shape(theta, (B, ansatz.P), "theta")
    if not per_row_system:  # one system for every row: [L] or [1, L]
        coeffs = coeffs.reshape(-1) if coeffs.dim() == 2 and coeffs.shape[0] == 1 else coeffs
        strings = strings.reshape(-1, 2) if strings.dim() == 3 and strings.shape[0] == 1 else strings
    _shape(coeffs, (B, Lt) if per_row_system else (Lt,), "coeffs")
    _shape(strings, (B, Lt, 2) if per_row_system else (Lt, 2), "strings")
    if out is None:
        C = torch.empty(B, dtype=torch.float64, device=theta.device)
        grad = torch.empty((B, ansatz.P), dtype=torch.float64, device=theta.device)
    else:
        C = _out(out[0], (B,), torch.float64, "C")
        grad = _out(out[1], (B, ansatz.P), torch.float64, "grad")
    bk, bt = _b_args(b_kind, b)
    a = ansatz.c()
    L.call("dvq_vqls_grad_adjoint", ctypes.byref(a), _p(theta), B, PRECISIONS[precision],
           _p(coeffs), _p(strings), Lt, int(per_row_system), bk, _p(bt), KINDS[kind], _p(C),
           _p(grad), _stream(theta))
    return C, grad


class AdjointCost(torch.autograd.Function):
    """C(theta) with the adjoint kernel's gradient as its backward."""

    @staticmethod
    def forward(ctx, theta, ansatz, coeffs, strings, kind, precision, b_kind, b):
        C, grad = vqls_grad_adjoint(ansatz, theta.detach(), coeffs, strings, kind, precision, b_kind, b)
        ctx.save_for_backward(grad)
        ctx.shape = theta.shape
        return C if theta.dim() > 1 else C[0]

    @staticmethod
    def backward(ctx, gC):
        (grad,) = ctx.saved_tensors
        g = grad * (gC.reshape(-1, 1) if gC.dim() > 0 else gC)
        return g.reshape(ctx.shape), None, None, None, None, None, None, None


def gd_step(theta: torch.Tensor, grad: torch.Tensor, lr: float) -> None:
    """theta -= lr * grad, in place (float64, contiguous, one size)."""
    _out(theta, tuple(theta.shape), torch.float64, "theta")
    _out(grad, tuple(grad.shape), torch.float64, "grad")
    if theta.numel() != grad.numel():
        raise ValueError(f"theta has {theta.numel()} elements, grad {grad.numel()}")
    L.call("dvq_gd_step", _p(theta), _p(grad), theta.numel(), float(lr), _stream(theta))


def fidelity(ansatz: AnsatzSpec, theta: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """|<target|V(theta)|0>|^2 per row, float64 [B]."""
    theta = _cuda(theta, torch.float64, "theta")
    if theta.dim() == 1:
        theta = theta.unsqueeze(0)
    target = _cuda(target, torch.complex128, "target")
    _shape(theta, (theta.shape[0], ansatz.P), "theta")
    _shape(target, (1 << ansatz.n,), "target")
    F = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    a = ansatz.c()
    L.call("dvq_fidelity", ctypes.byref(a), _p(theta), theta.shape[0], _p(target), _p(F), _stream(theta))
    return F


# -------------------------------------------------------------- warm-start MLP

def mlp_shape(d_in: int, hidden: int, d_out: int) -> L.MlpShape:
    return L.MlpShape(d_in, hidden, d_out)


def mlp_param_count(shape: L.MlpShape) -> int:
    return int(L.load().dvq_mlp_param_count(ctypes.byref(shape)))


def mlp_forward(shape: L.MlpShape, params: torch.Tensor, X: torch.Tensor, out=None):
    """(Y, H1, H2) float32; bfloat16 operands, float32 accumulation."""
    params = _cuda(params, torch.float32, "params")
    X = _cuda(X, torch.float32, "X")
    B = X.shape[0]
    _shape(params, (mlp_param_count(shape),), "params")
    _shape(X, (B, shape.d_in), "X")
    if out is None:
        H1 = torch.empty((B, shape.hidden), dtype=torch.float32, device=X.device)
        H2 = torch.empty_like(H1)
        Y = torch.empty((B, shape.d_out), dtype=torch.float32, device=X.device)
    else:
        Y = _out(out[0], (B, shape.d_out), torch.float32, "Y")
        H1 = _out(out[1], (B, shape.hidden), torch.float32, "H1")
        H2 = _out(out[2], (B, shape.hidden), torch.float32, "H2")
    L.call("dvq_mlp_forward", ctypes.byref(shape), _p(params), _p(X), B, _p(H1), _p(H2), _p(Y), _stream(X))
    return Y, H1, H2


def mlp_loss_grad(Y: torch.Tensor, T: torch.Tensor, out=None):
    """(dY float32, loss float64 [1]) of mean(1 - cos(Y - T))."""
    Y = _cuda(Y, torch.float32, "Y")
    T = _cuda(T, torch.float32, "T")
    _shape(T, tuple(Y.shape), "T")
    if out is None:
        dY = torch.empty_like(Y)
        loss = torch.empty(1, dtype=torch.float64, device=Y.device)
    else:
        dY = _out(out[0], tuple(Y.shape), torch.float32, "dY")
        loss = _out(out[1], (1,), torch.float64, "loss")
    L.call("dvq_mlp_loss_grad", _p(Y), _p(T), Y.numel(), _p(dY), _p(loss), _stream(Y))
    return dY, loss


def mlp_backward(shape: L.MlpShape, params, X, H1, H2, dY, workspace=None, out=None):
    """Parameter gradients, packed like params."""
    params = _cuda(params, torch.float32, "params")
    X, H1, H2, dY = (_cuda(t, torch.float32, nm) for t, nm in ((X, "X"), (H1, "H1"), (H2, "H2"), (dY, "dY")))
    B = X.shape[0]
    P = mlp_param_count(shape)
    _shape(params, (P,), "params")
    _shape(X, (B, shape.d_in), "X")
    _shape(H1, (B, shape.hidden), "H1")
    _shape(H2, (B, shape.hidden), "H2")
    _shape(dY, (B, shape.d_out), "dY")
    lib = L.load()
    if workspace is None:
        workspace = torch.empty(lib.dvq_mlp_workspace_bytes(ctypes.byref(shape), B), dtype=torch.uint8,
                                device=X.device)
    dparams = torch.empty_like(params) if out is None else _out(out, (P,), torch.float32, "out")
    L.call("dvq_mlp_backward", ctypes.byref(shape), _p(params), _p(X), _p(H1), _p(H2), _p(dY), B,
           _p(dparams), _p(workspace), workspace.numel(), _stream(X))
    return dparams


def adamw_step(params, grads, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
               eps: float = 1e-8, weight_decay: float = 0.0) -> None:
    """In place on params, m, v (float32, contiguous, one size)."""
    for buf, nm in ((params, "params"), (m, "m"), (v, "v")):
        _out(buf, tuple(params.shape), torch.float32, nm)
    grads = _shape(_cuda(grads, torch.float32, "grads"), tuple(params.shape), "grads")
    L.call("dvq_adamw_step", _p(params), _p(grads), _p(m), _p(v), params.numel(), int(t), float(lr),
           float(beta1), float(beta2), float(eps), float(weight_decay), _stream(params))


def feature_stats(X: torch.Tensor, out=None):
    """(mean [d], 1/std [d]) float32 of the rows of X [rows, d] (n - 1 denominator)."""
    X = _cuda(X, torch.float32, "X")
    if X.dim() != 2:
        raise ValueError(f"X must be [rows, d], got {tuple(X.shape)}")
    d = X.shape[1]
    if out is None:
        mean = torch.empty(d, dtype=torch.float32, device=X.device)
        isd = torch.empty(d, dtype=torch.float32, device=X.device)
    else:
        mean = _out(out[0], (d,), torch.float32, "mean")
        isd = _out(out[1], (d,), torch.float32, "inv_std")
    L.call("dvq_feature_stats", _p(X), X.shape[0], d, _p(mean), _p(isd), _stream(X))
    return mean, isd


def _stats_args(stats, d_in: int):
    if stats is None:
        return None, None
    mean, isd = (_cuda(t, torch.float32, nm) for t, nm in ((stats[0], "mean"), (stats[1], "inv_std")))
    _shape(mean, (d_in,), "mean")
    _shape(isd, (d_in,), "inv_std")
    return mean, isd


def mlp_predict(shape: L.MlpShape, params: torch.Tensor, X: torch.Tensor, stats=None, out=None):
    """Y [batch, d_out] float32 from one fused launch; `stats` = (mean, 1/std)
    standardises the inputs on the device."""
    params = _cuda(params, torch.float32, "params")
    X = _cuda(X, torch.float32, "X")
    B = X.shape[0]
    _shape(params, (mlp_param_count(shape),), "params")
    _shape(X, (B, shape.d_in), "X")
    mean, isd = _stats_args(stats, shape.d_in)
    Y = torch.empty((B, shape.d_out), dtype=torch.float32, device=X.device) if out is None else \
        _out(out, (B, shape.d_out), torch.float32, "Y")
    L.call("dvq_mlp_predict", ctypes.byref(shape), _p(params), _p(X), B, _p(mean), _p(isd), _p(Y), _stream(X))
    return Y


class TrainWorkspace:
    """Scratch memory of dvq_mlp_train_step for a batch size, allocated once."""

    def __init__(self, shape: L.MlpShape, batch: int, device):
        nbytes = L.load().dvq_mlp_train_workspace_bytes(ctypes.byref(shape), batch)
        self.batch = batch
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)


def mlp_train_step(shape: L.MlpShape, params, m, v, t: int, X, T, rows=None, batch: int | None = None,
                   stats=None, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                   weight_decay: float = 0.0, workspace: TrainWorkspace | None = None, loss=None, grads=None):
    """One fused training step (forward, loss, backward, AdamW) on the rows
    `rows` (int32 [batch], device) of X [*, d_in] and T [*, d_out]; params,
    m, v updated in place.  `loss` ([1] float64) and `grads` (packed like
    params) receive the minibatch loss and gradient when given."""
    n_par = mlp_param_count(shape)
    params, m, v = (_out(x, (n_par,), torch.float32, nm) for x, nm in ((params, "params"), (m, "m"), (v, "v")))
    X = _cuda(X, torch.float32, "X")
    T = _cuda(T, torch.float32, "T")
    if X.dim() != 2 or X.shape[1] != shape.d_in:
        raise ValueError(f"X must be [*, {shape.d_in}], got {tuple(X.shape)}")
    _shape(T, (X.shape[0], shape.d_out), "T")
    if rows is not None:
        rows = _cuda(rows, torch.int32, "rows")
        if rows.dim() != 1:
            raise ValueError("rows must be 1-D")
        batch = rows.shape[0]
    elif batch is None:
        batch = X.shape[0]
    if batch > X.shape[0] and rows is None:
        raise ValueError(f"batch {batch} > rows of X {X.shape[0]}")
    mean, isd = _stats_args(stats, shape.d_in)
    if workspace is None or workspace.batch < batch:
        workspace = TrainWorkspace(shape, batch, X.device)
    if loss is not None:
        loss = _out(loss, (1,), torch.float64, "loss")
    if grads is not None:
        grads = _out(grads, (n_par,), torch.float32, "grads")
    L.call("dvq_mlp_train_step", ctypes.byref(shape), _p(params), _p(m), _p(v), int(t), float(lr), float(beta1),
           float(beta2), float(eps), float(weight_decay), _p(X), _p(T), X.shape[0], _p(rows), int(batch), _p(mean), _p(isd),
           _p(grads), _p(loss), _p(workspace.buf), workspace.buf.numel(), _stream(X))
    return workspace
