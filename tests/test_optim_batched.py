"""Host-side batched L-BFGS (the warm-start family's optimizer) on problems
with known minimisers: per-row convex quadratics (closed-form minimiser
M^-1 b) and per-row Rosenbrock functions (minimiser at 1)."""
import numpy as np

from paper_2604_14435_amd.optim import lbfgs_batched


def test_quadratics_reach_their_closed_form_minimisers():
    rng = np.random.default_rng(0)
    B, P = 16, 12
    M = np.stack([(lambda Q: Q @ Q.T + (i + 1) * 0.1 * np.eye(P))(rng.normal(size=(P, P))) for i in range(B)])
    b = rng.normal(size=(B, P))

    def ev(x):
        Mx = np.einsum("bij,bj->bi", M, x)
        return 0.5 * np.einsum("bi,bi->b", x, Mx) - np.einsum("bi,bi->b", b, x), Mx - b

    x, f = lbfgs_batched(ev, np.zeros((B, P)), iters=200)
    want = np.linalg.solve(M, b[..., None])[..., 0]
    assert np.max(np.abs(x - want)) < 1e-6
    assert np.allclose(f, ev(want)[0], atol=1e-10)


def test_rosenbrock_rows_each_reach_one():
    rng = np.random.default_rng(1)

    def ev(x):
        a, c = x[:, :-1], x[:, 1:]
        f = np.sum(100 * (c - a ** 2) ** 2 + (1 - a) ** 2, axis=1)
        g = np.zeros_like(x)
        g[:, :-1] += -400 * a * (c - a ** 2) - 2 * (1 - a)
        g[:, 1:] += 200 * (c - a ** 2)
        return f, g

    x, f = lbfgs_batched(ev, rng.normal(size=(8, 6)) * 0.5, iters=500)
    assert np.max(np.abs(x - 1.0)) < 1e-8
    assert f.max() < 1e-16


def test_rows_are_independent():
    """A row's trajectory does not depend on the other rows of the batch."""
    rng = np.random.default_rng(2)
    P = 5
    A = rng.normal(size=(3, P, P))
    M = np.einsum("bij,bkj->bik", A, A) + np.eye(P)

    def ev(x):
        Mx = np.einsum("bij,bj->bi", M[: x.shape[0]], x)
        return 0.5 * np.einsum("bi,bi->b", x, Mx) + np.sum(np.cos(x), axis=1), Mx - np.sin(x)

    x0 = rng.normal(size=(3, P))
    xa, _ = lbfgs_batched(ev, x0, iters=30)
    xb, _ = lbfgs_batched(ev, x0[:1], iters=30)
    assert np.array_equal(xa[0], xb[0])
