"""ctypes binding of ``libdvq.so`` (the C ABI declared in include/dvq.h).

Only declarations: every function keeps its C name and signature.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdvq.so")


class Ansatz(ctypes.Structure):
    _fields_ = [("n", c_int32), ("layers", c_int32), ("entangler", c_int32)]


class MlpShape(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("hidden", c_int32), ("d_out", c_int32)]


DVQ_OK = 0
DVQ_EINVAL = -1
DVQ_ECAPACITY = -2
DVQ_ENOMEM = -3
DVQ_EDEVICE = -4
DVQ_EUNSUPPORTED = -5
DVQ_ENONFINITE = -6

DVQ_COST_GLOBAL, DVQ_COST_LOCAL = 0, 1
DVQ_ENT_CZ_LADDER, DVQ_ENT_CNOT_LADDER = 0, 1
DVQ_F64, DVQ_F32 = 0, 1
DVQ_B_PLUS, DVQ_B_VECTOR = 0, 1
DVQ_EXEC_LITERAL, DVQ_EXEC_GENERIC, DVQ_EXEC_SHARED = 0, 1, 2

_A = POINTER(Ansatz)
_M = POINTER(MlpShape)
_V = c_void_p

SIGNATURES = {
    "dvq_status_string": (c_char_p, [c_int32]),
    "dvq_last_error": (c_char_p, []),
    "dvq_version": (c_char_p, []),
    "dvq_decompose_workspace_bytes": (c_size_t, [c_int32]),
    "dvq_pauli_decompose_dense": (c_int32, [_V, c_int32, _V, _V, c_size_t, _V]),
    "dvq_pauli_decompose": (c_int32, [_V, c_int32, c_double, c_int64, _V, _V, c_int64,
                                      POINTER(c_int64), POINTER(c_double), _V, c_size_t, _V]),
    "dvq_decompose_batch_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "dvq_pauli_decompose_batch": (c_int32, [_V, c_int32, c_int32, c_int64, _V, _V, POINTER(c_double), _V,
                                            c_size_t, _V]),
    "dvq_pauli_sum_dense": (c_int32, [_V, _V, c_int32, c_int32, _V, _V]),
    "dvq_circuit_count": (c_int64, [c_int32, c_int32, c_int32]),
    "dvq_vqls_terms": (c_int32, [_A, _V, c_int32, c_int32, _V, c_int32, c_int32, _V, c_int32,
                                 c_int32, _V, _V, _V]),
    "dvq_vqls_terms_rhs": (c_int32, [_A, _V, c_int32, c_int32, _V, c_int32, c_int32, _V, c_int32,
                                     c_int32, _V, _V, _V]),
    "dvq_vqls_cost": (c_int32, [_V, c_int32, c_int32, c_int32, _V, _V, c_int32, _V, _V, _V]),
    "dvq_grad_shift_workspace_bytes": (c_size_t, [_A, c_int32, c_int32]),
    "dvq_vqls_grad_shift": (c_int32, [_A, _V, c_int32, _V, _V, c_int32, c_int32, _V, c_int32,
                                      _V, _V, _V, c_size_t, _V]),
    "dvq_grad_shift_noalloc_max_bytes": (c_size_t, []),
    "dvq_vqls_grad_shift_noalloc": (c_int32, [_A, _V, c_int32, _V, _V, c_int32, c_int32, _V, c_int32,
                                              _V, _V, _V]),
    "dvq_vqls_grad_adjoint": (c_int32, [_A, _V, c_int32, c_int32, _V, _V, c_int32, c_int32,
                                        c_int32, _V, c_int32, _V, _V, _V]),
    "dvq_gd_step": (c_int32, [_V, _V, c_int64, c_double, _V]),
    "dvq_fidelity": (c_int32, [_A, _V, c_int32, _V, _V, _V]),
    "dvq_mlp_param_count": (c_int64, [_M]),
    "dvq_mlp_workspace_bytes": (c_size_t, [_M, c_int32]),
    "dvq_mlp_forward": (c_int32, [_M, _V, _V, c_int32, _V, _V, _V, _V]),
    "dvq_mlp_loss_grad": (c_int32, [_V, _V, c_int64, _V, _V, _V]),
    "dvq_mlp_backward": (c_int32, [_M, _V, _V, _V, _V, _V, c_int32, _V, _V, c_size_t, _V]),
    "dvq_adamw_step": (c_int32, [_V, _V, _V, _V, c_int64, c_int32, c_float, c_float, c_float,
                                 c_float, c_float, _V]),
    "dvq_feature_stats": (c_int32, [_V, c_int32, c_int32, _V, _V, _V]),
    "dvq_mlp_predict": (c_int32, [_M, _V, _V, c_int32, _V, _V, _V, _V]),
    "dvq_mlp_train_workspace_bytes": (c_size_t, [_M, c_int32]),
    "dvq_mlp_train_step": (c_int32, [_M, _V, _V, _V, c_int32, c_float, c_float, c_float, c_float, c_float,
                                     _V, _V, c_int32, _V, c_int32, _V, _V, _V, _V, _V, c_size_t, _V]),
}

_lib = None


class DvqError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        super().__init__(f"{func}: status {status}: {detail}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libdvq.so once and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2604_14435_amd.build); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, func: str) -> None:
    if status != DVQ_OK:
        lib = load()
        raise DvqError(status, func, lib.dvq_last_error().decode())


def call(name: str, *args) -> int:
    """Call entry point ``name`` and raise DvqError on a non-OK status."""
    st = getattr(load(), name)(*args)
    check(st, name)
    return st
