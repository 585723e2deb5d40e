"""The FP64 network reference: backpropagation against central finite differences."""
import numpy as np

from oracle import mlp


def _random_problem(seed=0, n=300):
    rng = np.random.default_rng(seed)
    w = np.concatenate([[0.2, 1.7, -0.1, 0.6], rng.standard_normal(3 * mlp.H + 1)])
    L = rng.uniform(-1.5, 0.5, n)
    t = np.sin(2 * L) + 0.3 * L
    return w, L, t


def test_backprop_matches_finite_differences():
    w, L, t = _random_problem()
    _, g = mlp.loss_grad(w, L, t)
    fd = mlp.finite_difference_grad(w, L, t)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_loss_definition():
    w, L, t = _random_problem(1)
    y, mu = mlp.forward(w, L)
    a, b, m, s, *_ = mlp.unpack(w)
    assert np.allclose(mu, m + s * y)
    assert abs(mlp.loss(w, L, t) - np.mean((y - (t - m) / s) ** 2)) < 1e-15
    l2, _ = mlp.loss_grad(w, L, t)
    assert abs(l2 - mlp.loss(w, L, t)) < 1e-14


def test_dead_units_have_zero_gradient():
    w, L, t = _random_problem(2)
    # push unit 0 far negative: no sample activates it
    w[mlp.HDR + 0] = 1.0
    w[mlp.HDR + mlp.H + 0] = -100.0
    _, g = mlp.loss_grad(w, L, t)
    assert g[0] == 0 and g[mlp.H] == 0 and g[2 * mlp.H] == 0
