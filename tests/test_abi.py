"""The C-ABI library loads and exports every declared symbol; host-side
argument validation (no GPU needed: every call here fails before any HIP call)."""
import ctypes
import os
import re

import pytest

from paper_2604_14435_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dvq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dvq_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_bound_functions():
    assert set(declared_functions()) == set(L.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_version():
    lib = L.load()
    assert lib.dvq_version().decode().startswith("dvq")
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.dvq_status_string(s)
    assert b"unknown" in lib.dvq_status_string(42)


def test_circuit_counts_match_paper():
    lib = L.load()
    # 2(n+1)L^2 (Section II-B after Eq. (4)); global 2(L^2 + L)
    assert lib.dvq_circuit_count(10, 4, 1) == 352
    assert lib.dvq_circuit_count(10, 64, 1) == 90112
    assert lib.dvq_circuit_count(10, 128, 1) == 360448
    assert lib.dvq_circuit_count(10, 1024, 1) == 23068672
    assert lib.dvq_circuit_count(3, 8, 0) == 144
    assert lib.dvq_circuit_count(0, 8, 0) == 0


@pytest.mark.parametrize("n,layers,ent", [(0, 1, 0), (14, 1, 0), (3, 0, 0), (3, 1, 7)])
def test_terms_rejects_bad_ansatz(n, layers, ent):
    lib = L.load()
    a = L.Ansatz(n, layers, ent)
    st = lib.dvq_vqls_terms(ctypes.byref(a), None, 1, 0, None, 1, 0, None, 1, 0, None, None, None)
    assert st == L.DVQ_EINVAL


def test_terms_rejects_null_and_sizes():
    lib = L.load()
    a = L.Ansatz(3, 2, 0)
    dummy = ctypes.c_void_p(16)
    assert lib.dvq_vqls_terms(ctypes.byref(a), None, 1, 0, dummy, 8, 0, None, 0, 0, dummy, dummy, None) == L.DVQ_EINVAL
    assert lib.dvq_vqls_terms(ctypes.byref(a), dummy, 0, 0, dummy, 8, 0, None, 0, 0, dummy, dummy, None) == L.DVQ_EINVAL
    assert lib.dvq_vqls_terms(ctypes.byref(a), dummy, 1, 0, dummy, 0, 0, None, 0, 0, dummy, dummy, None) == L.DVQ_EINVAL
    # general b without the vector
    assert lib.dvq_vqls_terms(ctypes.byref(a), dummy, 1, 0, dummy, 8, 1, None, 0, 0, dummy, dummy, None) == L.DVQ_EINVAL
    # unknown execution mode
    assert lib.dvq_vqls_terms(ctypes.byref(a), dummy, 1, 0, dummy, 8, 0, None, 0, 9, dummy, dummy, None) == L.DVQ_EINVAL
    assert b"exec" in lib.dvq_last_error()


def test_terms_rhs_rejects_bad_input():
    lib = L.load()
    a = L.Ansatz(3, 2, 0)
    d = ctypes.c_void_p(16)
    f = lib.dvq_vqls_terms_rhs
    assert f(ctypes.byref(a), d, 1, 0, d, 8, 0, d, 0, 0, d, d, None) == L.DVQ_EINVAL  # R < 1
    assert f(ctypes.byref(a), d, 1, 0, d, 8, 65537, d, 0, 0, d, d, None) == L.DVQ_EINVAL  # R too large
    assert f(ctypes.byref(a), d, 1, 0, d, 8, 2, None, 0, 0, d, d, None) == L.DVQ_EINVAL  # no b
    assert f(ctypes.byref(a), d, 1, 0, d, 8, 2, d, 5, 0, d, d, None) == L.DVQ_EINVAL  # cost kind
    assert f(ctypes.byref(a), d, 1, 0, d, 8, 2, d, 0, 9, d, d, None) == L.DVQ_EINVAL  # exec
    assert b"exec" in lib.dvq_last_error()


def test_decompose_rejects_bad_input():
    lib = L.load()
    lout = ctypes.c_int64(-1)
    d = ctypes.c_void_p(16)
    assert lib.dvq_pauli_decompose(d, 0, 0.01, 0, d, d, 8, ctypes.byref(lout), None, d, 1 << 30, None) == L.DVQ_EINVAL
    assert lib.dvq_pauli_decompose(d, 13, 0.01, 0, d, d, 8, ctypes.byref(lout), None, d, 1 << 30, None) == L.DVQ_EINVAL
    assert lib.dvq_pauli_decompose(d, 4, -1.0, 0, d, d, 8, ctypes.byref(lout), None, d, 1 << 30, None) == L.DVQ_EINVAL
    assert lib.dvq_pauli_decompose(d, 4, float("nan"), 0, d, d, 8, ctypes.byref(lout), None, d, 1 << 30, None) == L.DVQ_EINVAL
    # workspace too small is a capacity error, reported before any launch
    assert lib.dvq_pauli_decompose(d, 4, 0.01, 0, d, d, 8, ctypes.byref(lout), None, d, 16, None) == L.DVQ_ECAPACITY
    assert lib.dvq_decompose_workspace_bytes(12) >= 8 * 4 ** 12
    assert lib.dvq_decompose_workspace_bytes(13) == 0


def test_decompose_batch_rejects_bad_input():
    lib = L.load()
    d = ctypes.c_void_p(16)
    f = (ctypes.c_double * 4)()
    big = 1 << 40
    assert lib.dvq_pauli_decompose_batch(d, 4, 0, 8, d, d, f, d, big, None) == L.DVQ_EINVAL  # B < 1
    assert lib.dvq_pauli_decompose_batch(d, 4, 4, 0, d, d, f, d, big, None) == L.DVQ_EINVAL  # top_L < 1
    assert lib.dvq_pauli_decompose_batch(d, 4, 4, 257, d, d, f, d, big, None) == L.DVQ_EINVAL  # > 4^n
    assert lib.dvq_pauli_decompose_batch(d, 4, 4, 8, d, d, None, d, big, None) == L.DVQ_EINVAL  # no error array
    assert lib.dvq_pauli_decompose_batch(d, 13, 4, 8, d, d, f, d, big, None) == L.DVQ_EINVAL
    need = lib.dvq_decompose_batch_workspace_bytes(4, 4)
    assert need > lib.dvq_decompose_workspace_bytes(4)
    assert lib.dvq_decompose_batch_workspace_bytes(4, 8) > need
    assert lib.dvq_pauli_decompose_batch(d, 4, 4, 8, d, d, f, d, need - 1, None) == L.DVQ_ECAPACITY


def test_grad_entry_points_reject_bad_input():
    lib = L.load()
    d = ctypes.c_void_p(16)
    a = L.Ansatz(3, 2, 0)
    assert lib.dvq_vqls_grad_adjoint(ctypes.byref(a), d, 0, 1, d, d, 8, 0, 0, None, 1, d, d, None) == L.DVQ_EINVAL
    assert lib.dvq_vqls_grad_adjoint(ctypes.byref(a), d, 1, 1, d, d, 8, 2, 0, None, 1, d, d, None) == L.DVQ_EINVAL
    need = lib.dvq_grad_shift_workspace_bytes(ctypes.byref(a), 8, 0)
    assert need > 0
    assert lib.dvq_vqls_grad_shift(ctypes.byref(a), d, 0, d, d, 8, 0, None, 0, d, d, d, need - 1, None) == L.DVQ_ECAPACITY
    # the entry point without a workspace: argument and scratch-size checks
    # come before any HIP call
    bad = L.Ansatz(3, 0, 0)
    assert lib.dvq_vqls_grad_shift_noalloc(ctypes.byref(bad), d, 0, d, d, 8, 0, None, 0, d, d, None) == L.DVQ_EINVAL
    assert lib.dvq_vqls_grad_shift_noalloc(ctypes.byref(a), d, 0, d, d, 8, 0, None, 0, None, d, None) == L.DVQ_EINVAL
    assert lib.dvq_vqls_grad_shift_noalloc(ctypes.byref(a), d, 0, d, d, 0, 0, None, 0, d, d, None) == L.DVQ_EINVAL
    big = L.Ansatz(10, 1, 0)
    assert lib.dvq_vqls_grad_shift_noalloc(ctypes.byref(big), d, 0, d, d, 512, 0, None, 1, d, d, None) == L.DVQ_ECAPACITY
    assert lib.dvq_grad_shift_noalloc_max_bytes() == 32 << 20
    assert lib.dvq_gd_step(None, d, 4, 0.1, None) == L.DVQ_EINVAL
    assert lib.dvq_gd_step(d, d, -1, 0.1, None) == L.DVQ_EINVAL


def test_binding_checks_shapes_before_any_launch():
    """The kernels index buffers by the sizes they are given: the binding
    rejects mismatched inputs and outputs before calling the library (the
    tensors are never touched, so CPU tensors stand in: the dtype/device
    check comes first and is what fires for them)."""
    torch = pytest.importorskip("torch")
    from paper_2604_14435_amd import api

    an = api.AnsatzSpec(3, 2, "cz")
    with pytest.raises(TypeError):
        api.vqls_terms(an, torch.zeros(1, 6, dtype=torch.float64), torch.zeros(2, 2, dtype=torch.int32))
    with pytest.raises(ValueError):
        api._shape(torch.zeros(1, 5), (1, 6), "theta")
    with pytest.raises(TypeError):
        api._out(torch.zeros(1, 6, dtype=torch.float64), (1, 6), torch.float64, "out")
    with pytest.raises(ValueError):
        api._square(torch.zeros(6, 6))
    api._square(torch.zeros(8, 8))
