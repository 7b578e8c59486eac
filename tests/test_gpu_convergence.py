"""GPU convergence: the L-BFGS-B driver on the GPU cost and gradient.

Mirrors the oracle's convergence pin (no pruning, RY + CNOT ladder, the
paper reports fidelity > 0.9999 at four qubits): the fast form (complex64
circuits for the cost, complex64 adjoint for the gradient) reaches
fidelity >= 0.9999 against the classical solution; the plain (complex128
shift rule) and complex128 adjoint forms agree evaluation by evaluation.
"""
import numpy as np
import pytest

from oracle import linalg as ola
from oracle import pauli as op
from workloads import plus_state, theta_uniform, toeplitz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2604_14435_amd import api  # noqa: E402
from paper_2604_14435_amd.optim import Evaluator, lbfgs, lbfgs_refine  # noqa: E402

DEV = "cuda:0"


def _unpruned(n, a, b):
    A = toeplitz(n, a, b)
    c, s, _ = api.pauli_decompose(torch.from_numpy(A).to(DEV), tau=0.0)
    assert c.shape[0] == 1 << n
    return A, c, s


@pytest.mark.parametrize("n,layers,kind", [(3, 2, "global"), (3, 2, "local"), (4, 4, "local")])
def test_fast_form_reaches_fidelity(n, layers, kind):
    A, c, s = _unpruned(n, 1.0, -0.4)
    an = api.AnsatzSpec(n, layers, "cnot")
    xsol = ola.solve(A, plus_state(n))
    ev = Evaluator(an, c, s, "f32", kind)
    best = 0.0
    for seed in range(4):
        th, tr = lbfgs(ev, theta_uniform(an.P, seed=seed), max_evals=1500)
        F = api.fidelity(an, torch.from_numpy(th).to(DEV).unsqueeze(0),
                         torch.from_numpy(xsol.astype(np.complex128)).to(DEV)).item()
        best = max(best, F)
        if best >= 0.9999:
            break
    assert best >= 0.9999


def test_plain_and_adjoint_forms_agree():
    """Same start, same first L-BFGS evaluations: the shift rule and the
    adjoint give the same cost and gradient in complex128."""
    A, c, s = _unpruned(3, 1.0, -0.4)
    an = api.AnsatzSpec(3, 2, "cnot")
    th0 = theta_uniform(an.P, seed=1)
    ep, ea = Evaluator(an, c, s, "f64", "local"), Evaluator(an, c, s, "f64-adjoint", "local")
    _, tp = lbfgs(ep, th0, max_evals=12)
    _, ta = lbfgs(ea, th0, max_evals=12)
    k = min(len(tp.costs), len(ta.costs))
    assert k >= 10
    assert np.max(np.abs(np.array(tp.costs[:k]) - np.array(ta.costs[:k]))) < 1e-10
    cp, gp = ep(th0)
    ca, ga = ea(th0)
    assert abs(cp - ca) < 1e-12 and np.max(np.abs(gp - ga)) < 1e-10


def test_target_stops_early():
    """A target equal to the lowest cost of the first six evaluations of an
    unconstrained run stops the (deterministic) rerun at that evaluation."""
    A, c, s = _unpruned(3, 1.0, -0.4)
    an = api.AnsatzSpec(3, 2, "cnot")
    ev = Evaluator(an, c, s, "f64-adjoint", "local")
    th0 = theta_uniform(an.P, seed=0)
    _, full = lbfgs(ev, th0, max_evals=500)
    assert full.evals > 6
    target = min(full.costs[:6])
    first = next(i for i, v in enumerate(full.costs) if v <= target)
    _, tr = lbfgs(ev, th0, max_evals=500, target=target)
    assert tr.stop == "target reached" and tr.evals == first + 1


def test_refinement_continues_after_float32_stalls():
    """n = 10, L = 64, RY + CNOT ladder from V|0> = b: complex64 L-BFGS stops
    in a flat region where its cost no longer resolves the steps; the
    complex128 phase of the mixed driver continues to a lower cost."""
    n = 10
    A = toeplitz(n, 1.0, -0.45)
    c, s, _ = api.pauli_decompose(torch.from_numpy(A).to(DEV), tau=0.01)
    an = api.AnsatzSpec(n, 4, "cnot")
    th0 = np.zeros(an.P)
    th0[:n] = np.pi / 2
    ev32, ev64 = Evaluator(an, c, s, "f32-adjoint"), Evaluator(an, c, s, "f64-adjoint")
    _, t32 = lbfgs(ev32, th0, max_evals=600, gtol=1e-12)
    assert t32.evals < 600  # stopped on its own
    th, tr = lbfgs_refine(ev32, ev64, th0, max_evals=600, gtol=1e-12)
    assert "float64" in tr.stop and tr.evals > t32.evals
    assert min(tr.costs) < min(t32.costs) - 1e-4
    assert len(tr.iter_evals) == len(tr.thetas) and tr.iter_evals == sorted(tr.iter_evals)
