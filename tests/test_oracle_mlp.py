"""Pins of the FP64 warm-start MLP reference (CPU only)."""
import numpy as np

from oracle import mlp as om


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3])
    got = om.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even mantissa (1.0);
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7
    assert got[3] == 1.0 + 2 ** -6 and got[4] == -2.5
    assert abs(got[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = om.init_params(2, 16, 5, seed=1)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((7, 2))
    t = rng.uniform(-3, 3, (7, 5))

    def L(pp):
        y, _ = om.forward(pp, X, bf16=False)
        return om.loss_and_grad_output(y, t)[0]

    y, cache = om.forward(p, X, bf16=False)
    _, dy = om.loss_and_grad_output(y, t)
    g = om.backward(p, cache, dy, bf16=False)
    h = 1e-6
    for k in om.LAYERS:
        flat = p[k].ravel()
        for i in range(0, flat.size, max(1, flat.size // 13)):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k].ravel()[i] += h
            lp = L(pp)
            pp[k].ravel()[i] -= 2 * h
            lm = L(pp)
            assert abs((lp - lm) / (2 * h) - g[k].ravel()[i]) < 1e-8


def test_adamw_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2, so the update is
    lr * (sign(g) * |g| / (|g| + eps) + wd * p)."""
    rng = np.random.default_rng(2)
    p = om.init_params(2, 8, 3, seed=3)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(vv) for k, vv in p.items()}
    p0 = {k: vv.copy() for k, vv in p.items()}
    om.adamw_step(p, g, m, v, 1, lr=1e-2, weight_decay=0.1)
    for k in om.LAYERS:
        want = p0[k] - 1e-2 * (g[k] / (np.abs(g[k]) + 1e-8) + 0.1 * p0[k])
        assert np.max(np.abs(p[k] - want)) < 1e-15
