"""GPU parity: cost assembly, parameter-shift and adjoint gradients, gradient
descent and fidelity vs the oracle.

Bars: cost within 1e-6 absolute (1e-12 in float64 where both sides are
float64 end to end); gradients: adjoint float64 == exact shift rule within
1e-10, float32 within 1e-5; trajectory theta within 1e-10 after 50 steps.
"""
import math

import numpy as np
import pytest

from oracle import circuit as qc
from oracle import cost as oc
from oracle import linalg as ola
from oracle import pauli as op
from workloads import plus_state, random_unit_vector, theta_uniform, toeplitz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _system(n, a, b, tau=None, top_L=None):
    A = toeplitz(n, a, b)
    C = op.decompose_fwht(A)
    keep = op.select_tau(C, tau) if tau is not None else op.select_top(C, top_L)
    c, xs, zs = op.kept_terms(C, keep)
    strings = np.stack([xs, zs], axis=1).astype(np.int32)
    At = op.reconstruct(c, xs, zs, n)
    return A, At, c, xs, zs, strings


@pytest.mark.parametrize("kind", ["global", "local"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cost_from_terms_small(kind, precision):
    n, layers = 3, 2
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, tau=0.01)
    th = theta_uniform(n * layers, seed=0)
    an = api.AnsatzSpec(n, layers, "cz")
    beta, other = api.vqls_terms(an, _gpu(th), _gpu(strings), kind, precision)
    C, parts = api.vqls_cost(_gpu(c), n, kind, beta, other)
    wb, wo = qc.terms(th, n, layers, "cz", xs, zs, kind)
    want = oc.cost_from_terms(c, wb, wo, n, kind)
    tol = 1e-12 if precision == "f64" else 1e-6
    assert abs(C.item() - want) < tol
    num, psi = oc.aggregate(c, wb, wo, kind)
    p = parts[0].cpu().numpy()
    assert abs(p[0] - num) < (1e-11 if precision == "f64" else 1e-5)
    assert abs(p[1] - psi) < (1e-11 if precision == "f64" else 1e-5)


def test_cost_n10_L64_both_precisions():
    """Cost of the full n = 10, L = 64 evaluation vs the dense definition."""
    n, layers = 10, 4
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.45, tau=0.01)
    th = theta_uniform(n * layers, seed=0)
    x = qc.ansatz_state(th, n, layers)
    want = oc.cost_dense(At, x, n, "local")
    an = api.AnsatzSpec(n, layers, "cz")
    for precision, tol in (("f64", 1e-12), ("f32", 1e-6)):
        beta, delta = api.vqls_terms(an, _gpu(th), _gpu(strings), "local", precision)
        C, _ = api.vqls_cost(_gpu(c), n, "local", beta, delta)
        assert abs(C.item() - want) < tol, precision


@pytest.mark.parametrize("kind", ["global", "local"])
def test_shift_rule_gradient_small(kind):
    n, layers = 3, 2
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, tau=0.01)
    th = theta_uniform(n * layers, seed=0)
    an = api.AnsatzSpec(n, layers, "cz")
    C, g = api.vqls_grad_shift(an, _gpu(th), _gpu(c), _gpu(strings), kind, "f64")
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", kind)
    C0, g0 = oc.grad_parameter_shift(parts, th, n, kind)
    assert abs(C.item() - C0) < 1e-12
    assert np.max(np.abs(g.cpu().numpy() - g0)) < 1e-10


@pytest.mark.parametrize("kind", ["global", "local"])
@pytest.mark.parametrize("ent", ["cz", "cnot"])
@pytest.mark.parametrize("b_kind", ["plus", "vector"])
def test_adjoint_matches_shift_rule_and_fd(kind, ent, b_kind):
    n, layers = 4, 3
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, top_L=12)
    b = random_unit_vector(1 << n, seed=8) if b_kind == "vector" else None
    th = theta_uniform(n * layers, seed=1)
    an = api.AnsatzSpec(n, layers, ent)
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, ent, kind, b_kind, b)
    C0, g0 = oc.grad_parameter_shift(parts, th, n, kind)
    gfd = oc.grad_finite_difference(lambda t: oc.cost_theta_dense(t, At, n, layers, ent, kind, b_kind, b), th)
    assert np.max(np.abs(g0 - gfd)) < 1e-7
    for precision, tol in (("f64", 1e-10), ("f32", 1e-5)):
        C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), kind, precision, b_kind,
                                     None if b is None else _gpu(b))
        assert abs(C.item() - C0) < (1e-12 if precision == "f64" else 1e-6)
        assert np.max(np.abs(g[0].cpu().numpy() - g0)) < tol, precision


def test_adjoint_n10_L128_six_layers():
    """n = 10, tau = 0.005 -> L = 128, 6 layers (60 parameters): adjoint vs the
    exact shift rule (dense route) and central differences (h = 1e-4)."""
    n, layers = 10, 6
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.45, tau=0.005)
    assert len(xs) == 128
    th = theta_uniform(n * layers, seed=0)
    an = api.AnsatzSpec(n, layers, "cz")
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "local")
    C0, g0 = oc.grad_parameter_shift(parts, th, n, "local")
    f = lambda t: oc.cost_theta_dense(t, At, n, layers, "cz", "local")
    gfd = oc.grad_finite_difference(f, th, 1e-4)
    assert np.max(np.abs(g0 - gfd)) < 1e-7
    for precision, tol in (("f64", 1e-10), ("f32", 1e-5)):
        C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), "local", precision)
        assert abs(C.item() - C0) < (1e-12 if precision == "f64" else 1e-6)
        assert np.max(np.abs(g[0].cpu().numpy() - g0)) < tol


def test_adjoint_per_row_systems():
    """B = 4 rows, each with its own Toeplitz system (the warm-start data path)."""
    n, layers = 5, 2
    rows = []
    for i, (a, b) in enumerate([(1.0, -0.3), (0.9, -0.45), (1.2, -0.1), (0.8, -0.2)]):
        rows.append(_system(n, a, b, top_L=16))
    coeffs = np.stack([r[2] for r in rows])
    strings = np.stack([r[5] for r in rows])
    th = theta_uniform(4 * n * layers, seed=3).reshape(4, -1)
    an = api.AnsatzSpec(n, layers, "cz")
    C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(coeffs), _gpu(strings), "local", "f64",
                                 per_row_system=True)
    for r in range(4):
        At = rows[r][1]
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "local")
        C0, g0 = oc.grad_parameter_shift(parts, th[r], n, "local")
        assert abs(C[r].item() - C0) < 1e-12
        assert np.max(np.abs(g[r].cpu().numpy() - g0)) < 1e-10


def test_gradient_descent_trajectory_small_workload():
    """n = 3 workload: 50 gradient-descent steps (eta = 0.1) with the
    shift-rule gradient of the global cost; theta after every step within
    1e-10 of the oracle's trajectory."""
    n, layers, eta, steps = 3, 2, 0.1, 50
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, tau=0.01)
    th0 = theta_uniform(n * layers, seed=0)
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "global")
    want, wcost = oc.gradient_descent(th0, lambda t: oc.grad_parameter_shift(parts, t, n, "global"), eta, steps)
    an = api.AnsatzSpec(n, layers, "cz")
    theta = _gpu(th0.copy())
    cg, sg = _gpu(c), _gpu(strings)
    ws = api.ShiftWorkspace(an, len(c), "global", DEV)
    for s in range(steps):
        C, g = api.vqls_grad_shift(an, theta, cg, sg, "global", "f64", workspace=ws)
        assert abs(C.item() - wcost[s]) < 1e-12
        api.gd_step(theta, g, eta)
        assert np.max(np.abs(theta.cpu().numpy() - want[s + 1])) < 1e-10, s


def test_fidelity_matches_oracle():
    n, layers = 6, 3
    rng = np.random.default_rng(0)
    th = rng.uniform(0, 2 * math.pi, size=(5, n * layers))
    target = random_unit_vector(1 << n, seed=2, complex_=True)
    an = api.AnsatzSpec(n, layers, "cnot")
    F = api.fidelity(an, _gpu(th), _gpu(target)).cpu().numpy()
    for r in range(5):
        x = qc.ansatz_state(th[r], n, layers, "cnot")
        assert abs(F[r] - ola.fidelity(x, target)) < 1e-13


def test_adjoint_autograd_function():
    n, layers = 3, 2
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, tau=0.01)
    th = _gpu(theta_uniform(n * layers, seed=0)).requires_grad_(True)
    an = api.AnsatzSpec(n, layers, "cz")
    C = api.AdjointCost.apply(th, an, _gpu(c), _gpu(strings), "local", "f64", "plus", None)
    (2.0 * C).backward()
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cz", "local")
    C0, g0 = oc.grad_parameter_shift(parts, th.detach().cpu().numpy(), n, "local")
    assert abs(C.item() - C0) < 1e-12
    assert np.max(np.abs(th.grad.cpu().numpy() - 2 * g0)) < 1e-10


@pytest.mark.parametrize("ent", ["cz", "cnot"])
@pytest.mark.parametrize("n,layers,kind,b_kind,precision", [
    (10, 3, "local", "vector", "f64"), (10, 5, "global", "plus", "f32"),
    (10, 2, "global", "vector", "f64"), (10, 1, "local", "plus", "f64"),
    (10, 4, "local", "plus", "f32"), (10, 6, "global", "plus", "f64"),
    (11, 2, "local", "plus", "f32"), (11, 3, "global", "vector", "f32"),
    (11, 4, "local", "vector", "f32"), (11, 1, "global", "plus", "f32")])
def test_register_adjoint_shapes(ent, n, layers, kind, b_kind, precision):
    """The wavefront adjoint (n = 10, 11, both ladders): both cost kinds,
    both state preparations, odd and even depths; vs the exact shift rule."""
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, top_L=12)
    b = random_unit_vector(1 << n, seed=n + layers) if b_kind == "vector" else None
    th = theta_uniform(n * layers, seed=layers)
    an = api.AnsatzSpec(n, layers, ent)
    parts = lambda t: oc.parts_theta_dense(t, At, n, layers, ent, kind, b_kind, b)
    C0, g0 = oc.grad_parameter_shift(parts, th, n, kind)
    C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), kind, precision, b_kind,
                                 None if b is None else _gpu(b))
    tol_c, tol_g = (1e-12, 1e-10) if precision == "f64" else (1e-6, 1e-5)
    assert abs(C.item() - C0) < tol_c
    assert np.max(np.abs(g[0].cpu().numpy() - g0)) < tol_g


@pytest.mark.parametrize("ent", ["cz", "cnot"])
def test_register_adjoint_per_row_batch(ent):
    """B = 5 rows with their own systems at n = 10 (the warm-start data path)."""
    n, layers = 10, 4
    rows = [_system(n, a, b, top_L=16) for a, b in [(1.0, -0.3), (0.9, -0.45), (1.2, -0.1), (0.8, -0.2), (1.1, -0.49)]]
    coeffs = np.stack([r[2] for r in rows])
    strings = np.stack([r[5] for r in rows])
    th = theta_uniform(5 * n * layers, seed=9).reshape(5, -1)
    an = api.AnsatzSpec(n, layers, ent)
    C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(coeffs), _gpu(strings), "local", "f64",
                                 per_row_system=True)
    for r in range(5):
        At = rows[r][1]
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, ent, "local")
        C0, g0 = oc.grad_parameter_shift(parts, th[r], n, "local")
        assert abs(C[r].item() - C0) < 1e-12
        assert np.max(np.abs(g[r].cpu().numpy() - g0)) < 1e-10


@pytest.mark.parametrize("layers", [4, 6, 8])
def test_register_adjoint_cnot_bench_system(layers):
    """The bench system (n = 10, L = 64) with the RY + CNOT ladder, the
    ansatz of the fidelity runs: complex64 and complex128 register adjoints
    against the exact shift rule on the dense cost, both cost kinds."""
    n = 10
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.45, tau=0.01)
    th = theta_uniform(n * layers, seed=11)
    an = api.AnsatzSpec(n, layers, "cnot")
    for kind in ("local", "global"):
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, "cnot", kind)
        C0, g0 = oc.grad_parameter_shift(parts, th, n, kind)
        for precision, tol_c, tol_g in (("f64", 1e-12, 1e-10), ("f32", 1e-6, 1e-5)):
            C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), kind, precision)
            assert abs(C.item() - C0) < tol_c, (kind, precision)
            assert np.max(np.abs(g[0].cpu().numpy() - g0)) < tol_g, (kind, precision)


@pytest.mark.parametrize("ent,precision,L", [("cz", "f64", 100), ("cnot", "f32", 100), ("cnot", "f64", 100),
                                            ("cz", "f32", 3), ("cnot", "f64", 1)])
def test_register_adjoint_string_counts(ent, precision, L):
    """The four wavefronts split the strings of each Pauli sum (a quarter
    each, read 64 per load, two per batch): L = 100 gives 25 per wavefront
    (a batch remainder), L = 3 and L = 1 leave wavefronts without strings;
    vs the exact shift rule, local and global cost."""
    n, layers = 10, 2
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, top_L=L)
    th = theta_uniform(n * layers, seed=5)
    an = api.AnsatzSpec(n, layers, ent)
    tol_c, tol_g = (1e-12, 1e-10) if precision == "f64" else (1e-6, 1e-5)
    for kind in ("local", "global"):
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, ent, kind)
        C0, g0 = oc.grad_parameter_shift(parts, th, n, kind)
        C, g = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), kind, precision)
        assert abs(C.item() - C0) < tol_c, kind
        assert np.max(np.abs(g[0].cpu().numpy() - g0)) < tol_g, kind


@pytest.mark.parametrize("ent,precision,b_kind", [("cz", "f64", "plus"), ("cnot", "f32", "vector"),
                                                  ("cnot", "f64", "plus")])
def test_register_adjoint_rows_independent_of_batch(ent, precision, b_kind):
    """Each row runs on four wavefronts (Pauli sums split, register phases
    redundant): a row's result has the same bits in a batch of 300 and of
    256, and sampled rows match the exact shift rule."""
    n, layers = 10, 4
    A, At, c, xs, zs, strings = _system(n, 1.0, -0.4, top_L=24)
    b = random_unit_vector(1 << n, seed=3) if b_kind == "vector" else None
    th = theta_uniform(300 * n * layers, seed=21).reshape(300, -1)
    an = api.AnsatzSpec(n, layers, ent)
    bb = None if b is None else _gpu(b)
    C1, g1 = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), "local", precision, b_kind, bb)
    C4, g4 = api.vqls_grad_adjoint(an, _gpu(th[:256]), _gpu(c), _gpu(strings), "local", precision, b_kind, bb)
    assert torch.equal(C1[:256], C4) and torch.equal(g1[:256], g4)
    tol_c, tol_g = (1e-12, 1e-10) if precision == "f64" else (1e-6, 1e-5)
    for r in (0, 255, 299):
        parts = lambda t: oc.parts_theta_dense(t, At, n, layers, ent, "local", b_kind, b)
        C0, g0 = oc.grad_parameter_shift(parts, th[r], n, "local")
        assert abs(C1[r].item() - C0) < tol_c
        assert np.max(np.abs(g1[r].cpu().numpy() - g0)) < tol_g
