"""FP64 CPU oracle of the l(t) surrogate network: a multilayer perceptron with
GELU hidden activations, a mean-squared-error loss, its gradient by the chain
rule, and the Adam update of Kingma & Ba (2015, Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written in plain numpy
in float64, layer by layer as the definitions read; it shares no code with the
GPU library.

Parameter layout (the same flat vector the library's mlp_get_params returns):
W1, b1, W2, b2, ..., with each W stored out x in, row-major.

Definitions:
    gelu(z)  = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
    layer l: z_l = a_l W_l^T + b_l,  a_{l+1} = gelu(z_l) for hidden layers,
             the last layer is affine
    loss     = mean over rows and outputs of (y_hat - y)^2
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

DIMS = (19, 256, 256, 256, 64)


def param_count(dims=DIMS) -> int:
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def unpack(params: np.ndarray, dims=DIMS):
    """Views (W, b) per layer into the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == param_count(dims)
    out, o = [], 0
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        W = p[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = p[o:o + n_out]
        o += n_out
        out.append((W, b))
    return out


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z), phi the standard normal density."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, X, dims=DIMS, keep: bool = False):
    """Network output for the rows of X; with keep=True also the layer inputs
    a_l and pre-activations z_l needed by the backward pass."""
    layers = unpack(params, dims)
    a = np.asarray(X, dtype=np.float64)
    acts, pres = [], []
    for i, (W, b) in enumerate(layers):
        acts.append(a)
        z = a @ W.T + b
        pres.append(z)
        a = gelu(z) if i + 1 < len(layers) else z
    return (a, acts, pres) if keep else a


def loss_grad(params, X, Y, dims=DIMS):
    """Mean-squared-error loss and its gradient with respect to the flat
    parameter vector (same layout)."""
    out, acts, pres = forward(params, X, dims, keep=True)
    Y = np.asarray(Y, dtype=np.float64)
    count = Y.size
    diff = out - Y
    loss = float(np.sum(diff * diff) / count)
    layers = unpack(params, dims)
    grads = []
    dz = 2.0 * diff / count                       # d loss / d z of the last layer
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        dW = dz.T @ acts[i]
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if i > 0:
            da = dz @ W                           # d loss / d a_i
            dz = da * gelu_grad(pres[i - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(p, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step t >= 1 (Kingma & Ba 2015, Algorithm 1).
    Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
