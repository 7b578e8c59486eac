"""GPU parity at the full n = 10, L = 64 evaluation, element by element.

Workload: tridiag(-0.45, 1, -0.45), N = 1024, b = |+>^10, tau = 0.01 -> L = 64
strings, 4 layers RY + CZ ladder (40 angles), local cost, theta ~ U[0, 2pi)
from seed 0: 2(n+1)L^2 = 90,112 Hadamard-test circuits (Section II-B after
Eq. (4)), each run gate by gate by the oracle in a pool of at most 16
processes and compared with the GPU's value of the same term.

Bars (absolute, per term): 1e-12 for complex128 state vectors, 1e-5 for
complex64.  The plain parameter-shift gradient (2P + 1 = 81 rows of the
whole evaluation) is compared with the oracle's exact shift rule on the
dense definition of the cost: 1e-10 in float64, 1e-5 in float32.
"""
import numpy as np
import pytest

import _oracle_pool
from oracle import cost as oc
from oracle import pauli as op
from workloads import theta_uniform, toeplitz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402

DEV = "cuda:0"
N_, LAYERS_ = 10, 4


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def system():
    C = op.decompose_fwht(toeplitz(N_, 1.0, -0.45))
    keep = op.select_tau(C, 0.01)
    c, xs, zs = op.kept_terms(C, keep)
    assert len(xs) == 64
    strings = np.stack([xs, zs], axis=1).astype(np.int32)
    th = theta_uniform(N_ * LAYERS_, seed=0)
    return c, xs, zs, strings, th


@pytest.fixture(scope="module")
def oracle_terms(system):
    c, xs, zs, strings, th = system
    print(f"[parity] oracle: all 90112 circuits of n=10 L=64 on {_oracle_pool.workers()} processes", flush=True)
    return _oracle_pool.local_terms(N_, LAYERS_, "cz", xs, zs, th)


@pytest.mark.parametrize("exec_", ["literal", "shared"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_every_term_n10_L64(system, oracle_terms, precision, exec_):
    """All 4,096 beta and 40,960 delta terms (90,112 circuits) against the
    oracle's circuits, in the launch configuration the benchmark times."""
    c, xs, zs, strings, th = system
    wb, wd = oracle_terms
    an = api.AnsatzSpec(N_, LAYERS_, "cz")
    beta, delta = api.vqls_terms(an, _gpu(th), _gpu(strings), "local", precision, exec_=exec_)
    gb = beta[0].cpu().numpy()
    gd = delta[0].cpu().numpy()
    tol = 1e-12 if precision == "f64" else 1e-5
    eb, ed = np.abs(gb - wb), np.abs(gd - wd)
    assert eb.max() < tol, (precision, exec_, float(eb.max()), np.unravel_index(eb.argmax(), eb.shape))
    assert ed.max() < tol, (precision, exec_, float(ed.max()), np.unravel_index(ed.argmax(), ed.shape))
    C, _ = api.vqls_cost(_gpu(c), N_, "local", beta, delta)
    want = oc.cost_from_terms(c, wb, wd, N_, "local")
    assert abs(C.item() - want) < (1e-12 if precision == "f64" else 1e-6)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_shift_rule_gradient_n10_L64(system, precision, tol):
    """dvq_vqls_grad_shift (81 rows x 90,112 circuits) against the oracle's
    exact shift rule on the dense cost (Psi = ||A x||^2, E = sum_j <A x|U_b
    Z_j U_b^dagger|A x>)."""
    c, xs, zs, strings, th = system
    At = op.reconstruct(c, xs, zs, N_)
    parts = lambda t: oc.parts_theta_dense(t, At, N_, LAYERS_, "cz", "local")
    C0, g0 = oc.grad_parameter_shift(parts, th, N_, "local")
    an = api.AnsatzSpec(N_, LAYERS_, "cz")
    C, g = api.vqls_grad_shift(an, _gpu(th), _gpu(c), _gpu(strings), "local", precision)
    assert abs(C.item() - C0) < (1e-12 if precision == "f64" else 1e-6)
    err = np.abs(g.cpu().numpy() - g0)
    assert err.max() < tol, (precision, float(err.max()), int(err.argmax()))


def test_adjoint_cost_equals_circuit_cost_n10_L64(system):
    """The fast iteration computes the cost twice: from the adjoint sweep
    (dense state, float32) and from the 90,112 circuits (float32); both are
    the same C_L of Section II-C stage iii."""
    c, xs, zs, strings, th = system
    an = api.AnsatzSpec(N_, LAYERS_, "cz")
    beta, delta = api.vqls_terms(an, _gpu(th), _gpu(strings), "local", "f32")
    Cc, _ = api.vqls_cost(_gpu(c), N_, "local", beta, delta)
    Ca, _ = api.vqls_grad_adjoint(an, _gpu(th), _gpu(c), _gpu(strings), "local", "f32")
    assert abs(Ca.item() - Cc.item()) < 1e-6


@pytest.fixture(scope="module")
def oracle_terms_cnot8(system):
    c, xs, zs, strings, _ = system
    th = theta_uniform(N_ * 8, seed=1)
    print(f"[parity] oracle: all 90112 circuits of n=10 L=64, CNOT ladder, 8 layers, on "
          f"{_oracle_pool.workers()} processes", flush=True)
    return th, _oracle_pool.local_terms(N_, 8, "cnot", xs, zs, th)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_every_term_cnot_8_layers_n10_L64(system, oracle_terms_cnot8, precision):
    """The ansatz of the time-to-fidelity runs (RY + CNOT ladder, 8 layers,
    80 angles) on the same system: all 90,112 circuits against the oracle's,
    and the cost."""
    c, xs, zs, strings, _ = system
    th, (wb, wd) = oracle_terms_cnot8
    an = api.AnsatzSpec(N_, 8, "cnot")
    beta, delta = api.vqls_terms(an, _gpu(th), _gpu(strings), "local", precision)
    tol = 1e-12 if precision == "f64" else 1e-5
    eb = np.abs(beta[0].cpu().numpy() - wb)
    ed = np.abs(delta[0].cpu().numpy() - wd)
    assert eb.max() < tol, (precision, float(eb.max()))
    assert ed.max() < tol, (precision, float(ed.max()))
    C, _ = api.vqls_cost(_gpu(c), N_, "local", beta, delta)
    assert abs(C.item() - oc.cost_from_terms(c, wb, wd, N_, "local")) < (1e-12 if precision == "f64" else 1e-6)
