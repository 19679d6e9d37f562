"""FP64 reference MLP for the learned initial guess (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring). The learned guess is
not part of the paper (the paper warm-starts GMRES from the previous time
step, Section 3.6); this module is the plain definition the GPU kernels are
checked against: a fully connected network

    h_0 = x,  h_k = silu(h_{k-1} W_k + b_k)  (k = 1..K-1),  y = h_{K-1} W_K + b_K,
    silu(z) = z / (1 + exp(-z)),

the mean-squared loss over a batch, its gradients by the chain rule, and one
Adam step (Kingma and Ba 2015, bias-corrected moments).

``rnd`` (optional, default the identity) is applied to both operands of
every matrix product, forward and backward; passing a BF16 rounding gives
the arithmetic of kernels that store those operands in BF16 and accumulate
in higher precision. Biases, pre-activations and the bias gradients are
never rounded.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init(sizes, seed=0):
    """Weights W_k [n_in, n_out] ~ N(0, 1/n_in) (Xavier-style), biases 0."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        params.append((rng.standard_normal((a, b)) / np.sqrt(a), np.zeros(b)))
    return params


def _ident(a):
    return a


def forward(params, x, rnd=None):
    """Returns (y, cache) where cache holds the pre-activations."""
    rnd = rnd or _ident
    h = np.asarray(x, dtype=np.float64)
    cache = [h]
    for k, (W, b) in enumerate(params):
        z = rnd(h) @ rnd(W) + b
        if k < len(params) - 1:
            cache.append(z)
            h = silu(z)
        else:
            h = z
    return h, cache


def loss(params, x, t, rnd=None):
    """0.5 * mean over the batch of ||y - t||^2."""
    y, _ = forward(params, x, rnd)
    return 0.5 * np.sum((y - t) ** 2) / x.shape[0]


def backward(params, x, t, rnd=None):
    """Gradients of `loss` with respect to every W_k, b_k (chain rule)."""
    rnd = rnd or _ident
    y, cache = forward(params, x, rnd)
    B = x.shape[0]
    g = (y - t) / B  # dL/dy
    grads = [None] * len(params)
    hs = [cache[0]] + [silu(z) for z in cache[1:]]
    for k in range(len(params) - 1, -1, -1):
        W, _ = params[k]
        h_in = hs[k]
        grads[k] = (rnd(h_in).T @ rnd(g), g.sum(axis=0))
        if k > 0:
            g = (rnd(g) @ rnd(W).T) * silu_grad(cache[k])
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(t, m, v) (created if empty)."""
    if not state:
        state.update(t=0, m=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                     v=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
    state["t"] += 1
    t = state["t"]
    out = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][k][j] * b1 + (1 - b1) * g
            v = state["v"][k][j] * b2 + (1 - b2) * g * g
            state["m"][k] = tuple(m if i == j else state["m"][k][i] for i in range(2))
            state["v"][k] = tuple(v if i == j else state["v"][k][i] for i in range(2))
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out
