"""Pins for the FP64 surrogate oracle: central finite differences of the loss (backward pass),
the least-squares closed form (a network without hidden layers trained with Adam converges to
numpy.linalg.lstsq), Adam's first-step closed form, the SiLU derivative, and the ensemble's
de-normalised mean and (population) variance worked out by hand for three linear members."""
import numpy as np
import pytest

from oracle import surrogate as S
from synth.surrogate import init_params, regression_data


def test_silu_derivative_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (S.silu(z + h) - S.silu(z - h)) / (2 * h)
    assert np.allclose(S.silu_grad(z), fd, rtol=1e-8, atol=1e-10)
    assert S.silu(0.0) == 0.0 and S.silu_grad(0.0) == 0.5


def test_backward_matches_finite_differences():
    dims = S.layer_dims(7, 12, 3, 4)
    p = init_params(dims, seed=3)
    p += 0.05 * np.random.default_rng(0).standard_normal(p.size)     # non-zero biases
    X, Y = regression_data(9, 7, 4, seed=5)
    Yp, cache = S.forward(p, dims, X)
    loss, dY = S.mse(Yp, Y)
    g = S.backward(cache, dY)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k in rng.choice(p.size, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (S.mse(S.forward(pp, dims, X)[0], Y)[0] - S.mse(S.forward(pm, dims, X)[0], Y)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-9)


def test_linear_network_converges_to_least_squares():
    dims = S.layer_dims(5, 0, 0, 3)            # no hidden layer: y = x W + b
    rng = np.random.default_rng(2)
    X = rng.standard_normal((200, 5))
    Y = X @ rng.standard_normal((5, 3)) + 0.3 + 0.1 * rng.standard_normal((200, 3))
    p = init_params(dims, seed=1)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for t in range(1, 4001):
        Yp, cache = S.forward(p, dims, X)
        _, dY = S.mse(Yp, Y)
        p, m, v = S.adam(p, S.backward(cache, dY), m, v, t, lr=0.01 if t < 3000 else 0.001)
    Xa = np.hstack([X, np.ones((200, 1))])
    sol = np.linalg.lstsq(Xa, Y, rcond=None)[0]
    Ws, bs = S.unflatten(p, dims)
    assert np.abs(Ws[0] - sol[:5]).max() < 2e-3 and np.abs(bs[0] - sol[5]).max() < 2e-3


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    p = np.ones(4)
    p1, m, v = S.adam(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected m/sqrt(v) = g/|g| on the first step: each parameter moves by lr against sign(g)
    assert np.allclose(p1[:3], 1.0 - 0.01 * np.sign(g[:3]), rtol=0, atol=1e-7)
    assert p1[3] == 1.0


def test_ensemble_statistics():
    dims = S.layer_dims(4, 8, 2, 2)
    params = [init_params(dims, seed=7, member=k) for k in range(3)]
    X = np.random.default_rng(0).standard_normal((5, 4))
    mu, var = S.ensemble_predict(params, dims, X, 0.0, 1.0, 0.0, 1.0)
    outs = np.stack([S.forward(p, dims, X)[0] for p in params])
    assert np.allclose(mu, outs.mean(0)) and np.allclose(var, outs.var(0))
    same_mu, same_var = S.ensemble_predict([params[0]] * 3, dims, X, 0.0, 1.0, 0.0, 1.0)
    assert np.allclose(same_var, 0.0)


def test_ensemble_denormalisation_closed_form():
    """Three members without hidden layers (y_n = x_n W + b), worked by hand.  The raw input
    (3, -1) with x_mu = (1, 1), x_sd = (2, 4) normalises to (1, -0.5); the members then give
    normalised outputs (1, -0.5), (2, 0) and (3, 0.5): per component mean (2, 0) and population
    variance (2/3, 1/6).  De-normalising with y_mu = (10, -5), y_sd = (2, 3) shifts the mean to
    (10 + 2 * 2, -5 + 3 * 0) = (14, -5) and scales the variance by y_sd^2 to (8/3, 3/2)."""
    dims = S.layer_dims(2, 0, 0, 2)
    members = [
        (np.array([[1.0, 0.0], [0.0, 1.0]]), np.array([0.0, 0.0])),
        (np.array([[2.0, 0.0], [0.0, 2.0]]), np.array([0.0, 1.0])),
        (np.array([[3.0, 0.0], [0.0, 0.0]]), np.array([0.0, 0.5])),
    ]
    params = [S.flatten([W], [b]) for W, b in members]
    X = np.array([[3.0, -1.0]])
    mu, var = S.ensemble_predict(params, dims, X, np.array([1.0, 1.0]), np.array([2.0, 4.0]),
                                 np.array([10.0, -5.0]), np.array([2.0, 3.0]))
    assert np.allclose(mu, [[14.0, -5.0]], rtol=0, atol=1e-12)
    assert np.allclose(var, [[8.0 / 3.0, 1.5]], rtol=0, atol=1e-12)
