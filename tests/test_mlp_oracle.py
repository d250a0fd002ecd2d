"""Pins of the float64 oracle of the learned index's training loss.

The gradient is checked against central finite differences of the loss (a
derivative, not a retyping of the chain rule), against closed forms of the
special case w2 = 0, and the loss against its value at zero parameters.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as mo


def sample(seed, n=257, hidden=mo.HIDDEN):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 1.0, 3 * hidden + 1)
    x = rng.uniform(0.0, 1.0, n)
    y = np.sort(rng.uniform(0.0, 1.0, n))
    return p, x, y


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("hidden", [1, 3, mo.HIDDEN])
def test_gradient_matches_finite_differences(seed, hidden):
    p, x, y = sample(seed, hidden=hidden)
    _, g = mo.loss_and_grad(p, x, y, hidden)
    h = 1e-6
    fd = np.empty_like(p)
    for t in range(len(p)):
        e = np.zeros_like(p)
        e[t] = h
        fd[t] = (mo.loss(p + e, x, y, hidden) - mo.loss(p - e, x, y, hidden)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_loss_value_matches_definition_on_a_tiny_case():
    # H = 1, two samples, worked by hand: f(x) = 0.5 + 2 tanh(x - 1)
    p = np.array([1.0, -1.0, 2.0, 0.5])
    x = np.array([1.0, 2.0])
    y = np.array([0.0, 1.0])
    f = np.array([0.5, 0.5 + 2 * np.tanh(1.0)])
    want = ((f[0] - 0.0) ** 2 + (f[1] - 1.0) ** 2) / 2
    assert mo.loss(p, x, y, hidden=1) == pytest.approx(want, rel=1e-15)


def test_zero_output_weights_reduce_to_a_constant_model():
    p, x, y = sample(5)
    H = mo.HIDDEN
    p[2 * H:3 * H] = 0.0  # w2 = 0: f is the constant b2
    b2 = p[3 * H]
    loss, g = mo.loss_and_grad(p, x, y)
    assert loss == pytest.approx(np.mean((b2 - y) ** 2), rel=1e-12)
    # no signal reaches the first layer
    assert np.all(g[:2 * H] == 0.0)
    # d/d b2 = 2 mean(b2 - y); d/d w2[j] = 2 mean((b2 - y) tanh(w1 x + b1))
    assert g[3 * H] == pytest.approx(2 * np.mean(b2 - y), rel=1e-12)
    hj = np.tanh(np.outer(x, p[:H]) + p[H:2 * H])
    np.testing.assert_allclose(g[2 * H:3 * H], 2 * ((b2 - y) @ hj) / len(x), rtol=1e-12)


def test_zero_parameters_give_mean_square_of_targets():
    _, x, y = sample(7)
    assert mo.loss(np.zeros(mo.PARAMS), x, y) == pytest.approx(np.mean(y * y), rel=1e-15)


def test_gradient_vanishes_at_a_perfect_fit():
    p, x, _ = sample(9)
    y = mo.forward(p, x)
    loss, g = mo.loss_and_grad(p, x, y)
    assert loss == 0.0
    assert np.all(np.abs(g) < 1e-15)
