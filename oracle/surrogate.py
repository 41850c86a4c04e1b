"""FP64 numpy reference of the learned stress surrogate: a multilayer perceptron mapping a
normalised deformation history to normalised stress, its MSE loss, hand-written backward pass
and the Adam update (Kingma & Ba, ICLR 2015).  Test infrastructure only.

Parameter layout (shared interface with the GPU library, one ensemble member, FP32 or FP64):
for each layer l = 0..L-1 with fan-in d_l and fan-out d_{l+1}: W_l as a d_l x d_{l+1} row-major
block (x_{l+1} = x_l W_l + b_l), then b_l (d_{l+1}).  Hidden layers use SiLU, the last layer is linear.
"""
import numpy as np


def layer_dims(din, width, depth, dout):
    return [din] + [width] * depth + [dout]


def n_params(dims):
    return sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))


def unflatten(p, dims):
    Ws, bs, o = [], [], 0
    for l in range(len(dims) - 1):
        a, b = dims[l], dims[l + 1]
        Ws.append(p[o:o + a * b].reshape(a, b)); o += a * b
        bs.append(p[o:o + b]); o += b
    return Ws, bs


def flatten(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, dims, X):
    """Return (output, cache) for normalised inputs X [B, din]."""
    Ws, bs = unflatten(np.asarray(p, np.float64), dims)
    a = np.asarray(X, np.float64)
    acts, zs = [a], []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = a @ W + b
        zs.append(z)
        a = silu(z) if l < len(Ws) - 1 else z
        acts.append(a)
    return a, (Ws, acts, zs)


def mse(Yp, Y):
    """Mean over batch and components of (Yp - Y)^2, and its gradient with respect to Yp."""
    d = Yp - Y
    return float((d * d).mean()), 2.0 * d / d.size


def backward(cache, dY):
    """Gradient of the loss with respect to the flat parameters, given dLoss/dOutput."""
    Ws, acts, zs = cache
    gW, gb = [None] * len(Ws), [None] * len(Ws)
    dz = dY
    for l in range(len(Ws) - 1, -1, -1):
        gW[l] = acts[l].T @ dz
        gb[l] = dz.sum(0)
        if l > 0:
            dz = (dz @ Ws[l].T) * silu_grad(zs[l - 1])
    return flatten(gW, gb)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def normalise(X, mu, sd):
    return (X - mu) / sd


def ensemble_predict(params, dims, X, x_mu, x_sd, y_mu, y_sd):
    """Mean and variance over members of the de-normalised outputs for raw inputs X."""
    Xn = normalise(np.asarray(X, np.float64), x_mu, x_sd)
    outs = np.stack([forward(p, dims, Xn)[0] * y_sd + y_mu for p in params])
    return outs.mean(0), outs.var(0)
