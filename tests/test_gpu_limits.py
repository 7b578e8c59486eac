"""GPU runs at the documented size limits (through the C ABI).

Circuits at the largest state the LDS circuit kernel holds (n = 12 with
complex128, n = 13 with complex64: 128 KiB of amplitudes per workgroup),
the adjoint at n = 12 in complex64 against the exact shift rule, the
documented refusal of the complex128 adjoint at n = 12 (three LDS vectors,
192 KiB > 160 KiB), and top-L selection on a dense 4096 x 4096 matrix.
"""
import numpy as np
import pytest

from oracle import circuit as qc
from oracle import pauli as op
from workloads import random_symmetric, theta_uniform

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402
from paper_2604_14435_amd import _lib as L  # noqa: E402

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("n,precision,ent,tol", [(12, "f64", "cz", 1e-12), (13, "f32", "cnot", 1e-5)])
def test_largest_circuits(n, precision, ent, tol):
    rng = np.random.default_rng(n)
    N = 1 << n
    strings = rng.integers(0, N, size=(2, 2)).astype(np.int32)
    an = api.AnsatzSpec(n, 1, ent)
    th = theta_uniform(an.P, seed=n)
    beta, delta = api.vqls_terms(an, _gpu(th), _gpu(strings), "local", precision)
    beta, delta = beta[0].cpu().numpy(), delta[0].cpu().numpy()
    for l, m, j in ((0, 1, 0), (1, 0, n - 1), (1, 1, n // 2)):
        sl, sm = (int(strings[l, 0]), int(strings[l, 1])), (int(strings[m, 0]), int(strings[m, 1]))
        assert abs(beta[l, m] - qc.beta_term(th, n, 1, ent, sl, sm)) < tol
        assert abs(delta[j, l, m] - qc.delta_term(th, n, 1, ent, sl, sm, j)) < tol


def test_adjoint_n12_f32_matches_shift_rule():
    n = 12
    rng = np.random.default_rng(3)
    N = 1 << n
    strings = _gpu(rng.integers(0, N, size=(2, 2)).astype(np.int32))
    coeffs = _gpu(np.array([0.8 + 0.0j, -0.3 + 0.0j]))
    an = api.AnsatzSpec(n, 1, "cz")
    th = _gpu(theta_uniform(an.P, seed=4))
    Cs, gs = api.vqls_grad_shift(an, th, coeffs, strings, "local", "f32")
    Ca, ga = api.vqls_grad_adjoint(an, th, coeffs, strings, "local", "f32")
    assert abs(Ca.item() - Cs.item()) < 1e-6
    assert torch.max(torch.abs(ga[0] - gs)).item() < 1e-5


def test_adjoint_n12_f64_is_refused():
    n = 12
    strings = _gpu(np.array([[1, 2], [3, 0]], dtype=np.int32))
    coeffs = _gpu(np.array([1.0 + 0.0j, 0.5 + 0.0j]))
    an = api.AnsatzSpec(n, 1, "cz")
    th = _gpu(theta_uniform(an.P, seed=0))
    with pytest.raises(L.DvqError) as e:
        api.vqls_grad_adjoint(an, th, coeffs, strings, "local", "f64")
    assert e.value.status == L.DVQ_EUNSUPPORTED


def test_top_L_dense_n12():
    n, L_ = 12, 3000
    A = random_symmetric(n, seed=2)
    C = op.decompose_fwht(A)
    keep = op.select_top(C, L_)
    mag = np.sort(np.abs(C.ravel()))[::-1]
    assert mag[L_ - 1] - mag[L_] > 1e-15  # the cut is not an exact tie
    c, s, ferr = api.pauli_decompose(_gpu(A), top_L=L_)
    flat = s.cpu().numpy().astype(np.int64)
    assert np.array_equal(flat[:, 0] * (1 << n) + flat[:, 1], keep)
    assert np.max(np.abs(c.cpu().numpy() - C.ravel()[keep])) < 1e-13
    assert abs(ferr - op.frobenius_error(C, keep, A)) < 1e-12
