"""The fast iteration replayed from HIP graphs equals the same launches run
eagerly, replay by replay (with eager work and synchronisations between the
replays): the angles after every step bit for bit, and the last cost."""
import numpy as np
import pytest

from workloads import random_unit_vector, theta_uniform, toeplitz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402
from paper_2604_14435_amd.graphs import FastGradientDescent  # noqa: E402

DEV = "cuda:0"


def _eager_step(an, coeffs, strings, theta, eta, kind, b_kind, b):
    _, g = api.vqls_grad_adjoint(an, theta, coeffs, strings, kind, "f32", b_kind=b_kind, b=b)
    api.gd_step(theta, g, eta)


@pytest.mark.parametrize("n,layers,ent,kind,b_kind", [(10, 4, "cz", "local", "plus"), (10, 3, "cnot", "local", "vector"),
                                                      (4, 2, "cz", "global", "vector")])
def test_graph_steps_equal_eager_steps(n, layers, ent, kind, b_kind):
    A = torch.from_numpy(toeplitz(n, 1.0, -0.45)).to(DEV)
    coeffs, strings, _ = api.pauli_decompose(A, tau=0.01)
    an = api.AnsatzSpec(n, layers, ent)
    b = torch.from_numpy(random_unit_vector(1 << n, seed=5)).to(DEV) if b_kind == "vector" else None
    eta = 0.5
    th0 = torch.from_numpy(theta_uniform(an.P, seed=1)).to(DEV).view(1, -1)
    theta = th0.clone()
    fg = FastGradientDescent(an, coeffs, strings, theta, eta, kind, b_kind, b)
    assert torch.equal(theta, th0)  # building the graphs does not touch theta
    ref = th0.clone()
    for r in range(5):
        fg.step(1 + (r % 2))  # odd and even counts
        torch.cuda.synchronize()
        for _ in range(1 + (r % 2)):
            _eager_step(an, coeffs, strings, ref, eta, kind, b_kind, b)
        torch.cuda.synchronize()
        assert torch.equal(theta, ref), r
    # the last iteration's cost: at the angles before its update
    prev = ref.clone()
    _, g = api.vqls_grad_adjoint(an, prev, coeffs, strings, kind, "f32", b_kind=b_kind, b=b)
    fg.step(1)
    C = fg.last_cost().item()
    beta, other = api.vqls_terms(an, prev, strings, kind, "f32", b_kind=b_kind, b=b)
    want = api.vqls_cost(coeffs, n, kind, beta, other)[0].item()
    assert C == want
    assert np.isfinite(C)


@pytest.mark.parametrize("unroll", [2, 5])
def test_unrolled_graphs_equal_single_step_graphs(unroll):
    """Runs of `unroll` iterations captured as one graph give the angles and
    the cost of the single-iteration graphs, bit for bit, for step counts
    that start runs at both parities and leave remainders."""
    n = 10
    A = torch.from_numpy(toeplitz(n, 1.0, -0.45)).to(DEV)
    coeffs, strings, _ = api.pauli_decompose(A, tau=0.01)
    an = api.AnsatzSpec(n, 4, "cz")
    th0 = torch.from_numpy(theta_uniform(an.P, seed=3)).to(DEV).view(1, -1)
    one = FastGradientDescent(an, coeffs, strings, th0.clone(), 0.5)
    many = FastGradientDescent(an, coeffs, strings, th0.clone(), 0.5, unroll=unroll)
    for count in (1, unroll, unroll + 1, 2 * unroll + 3):
        one.step(count)
        many.step(count)
        torch.cuda.synchronize()
        assert one.k == many.k
        assert torch.equal(one.theta, many.theta), count
        assert one.last_cost().item() == many.last_cost().item()
    with pytest.raises(ValueError):
        FastGradientDescent(an, coeffs, strings, th0.clone(), 0.5, unroll=0)


@pytest.mark.parametrize("n,layers,form", [(10, 4, "f32"), (10, 3, "f32-adjoint"), (4, 2, "f64"), (4, 2, "f64-adjoint")])
def test_evaluator_graph_replays_equal_eager_calls(n, layers, form):
    """The L-BFGS evaluator replaying its HIP graph returns what eager
    launches return, call after call, for changing angles."""
    from paper_2604_14435_amd.optim import Evaluator

    A = torch.from_numpy(toeplitz(n, 1.0, -0.45)).to(DEV)
    coeffs, strings, _ = api.pauli_decompose(A, tau=0.01)
    an = api.AnsatzSpec(n, layers, "cz")
    eg = Evaluator(an, coeffs, strings, form, graph=True)
    ee = Evaluator(an, coeffs, strings, form, graph=False)
    rng = np.random.default_rng(7)
    th = theta_uniform(an.P, seed=2)
    for i in range(6):
        cg, gg = eg(th)
        ce, ge = ee(th)
        assert cg == ce and np.array_equal(gg, ge), i
        th = th - 0.1 * ge + 0.01 * rng.standard_normal(an.P)
    assert eg.graph is not None and ee.graph is None
