"""Seeded inputs for the stress surrogate: initial network parameters (Glorot uniform weights, zero
biases) in the flat per-member layout, and synthetic regression data for tests."""
import numpy as np

from .rng import generator


def init_params(dims, seed, member=0):
    rng = generator(seed, member)
    chunks = []
    for l in range(len(dims) - 1):
        a, b = dims[l], dims[l + 1]
        lim = np.sqrt(6.0 / (a + b))
        chunks.append(rng.uniform(-lim, lim, a * b))
        chunks.append(np.zeros(b))
    return np.concatenate(chunks)


def regression_data(n, din, dout, seed, noise=0.0):
    """Inputs ~ N(0, 1); targets a smooth nonlinear map of them (for training tests)."""
    rng = generator(seed, 0)
    X = rng.standard_normal((n, din))
    A = rng.standard_normal((din, dout)) / np.sqrt(din)
    B = rng.standard_normal((din, dout)) / np.sqrt(din)
    Y = X @ A + 0.5 * np.tanh(X @ B) + noise * rng.standard_normal((n, dout))
    return X, Y
