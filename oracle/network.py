"""FP64 reference of the warm-start network: a stack of circular 1D
convolutions (kernel 5) with tanh-approximated GELU between layers, applied
along the affected points of one body ordered around it.

Layout: X[b, l, c] (sequence, position, channel); weights W[tap * c_in + ci, co],
tap = 0..4 reads position (l + tap - 2) mod L; bias b[co].
    conv(X)[b, l, co] = sum_tap sum_ci W[tap*c_in+ci, co] X[b, (l+tap-2) mod L, ci] + bias[co]
Loss: mean over all (b, l) of (Y - T)^2 with a single output channel.
Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

C_GELU = np.sqrt(2.0 / np.pi)
A_GELU = 0.044715
TAPS = 5


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + A_GELU * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C_GELU * (z + A_GELU * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3.0 * A_GELU * z * z)


def conv1d(X, W, bias):
    B, L, cin = X.shape
    out = np.zeros((B, L, W.shape[1])) + bias[None, None, :]
    for tap in range(TAPS):
        Xs = np.roll(X, -(tap - 2), axis=1)          # Xs[:, l] = X[:, (l + tap - 2) mod L]
        out += Xs @ W[tap * cin:(tap + 1) * cin, :]
    return out


def conv1d_backward(X, W, dZ):
    B, L, cin = X.shape
    dX = np.zeros_like(X)
    dW = np.zeros_like(W)
    for tap in range(TAPS):
        Wt = W[tap * cin:(tap + 1) * cin, :]
        Xs = np.roll(X, -(tap - 2), axis=1)
        dW[tap * cin:(tap + 1) * cin, :] = np.einsum("blc,blo->co", Xs, dZ)
        dX += np.roll(dZ @ Wt.T, tap - 2, axis=1)     # position (l + tap - 2) receives dZ[l]
    db = dZ.sum(axis=(0, 1))
    return dX, dW, db


def init_params(sizes, seed):
    """He-style uniform initialisation, sizes = [c_in, width, ..., 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for cin, cout in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (TAPS * cin))
        params.append((rng.uniform(-lim, lim, size=(TAPS * cin, cout)), np.zeros(cout)))
    return params


def forward(params, X):
    acts = [X]
    pre = []
    h = X
    for li, (W, b) in enumerate(params):
        z = conv1d(h, W, b)
        pre.append(z)
        h = gelu(z) if li < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss_and_grads(params, X, T):
    Y, (acts, pre) = forward(params, X)
    diff = Y[..., 0] - T
    loss = np.mean(diff ** 2)
    dY = (2.0 / diff.size) * diff[..., None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        dZ = dY if li == len(params) - 1 else dY * gelu_grad(pre[li])
        dX, dW, db = conv1d_backward(acts[li], W, dZ)
        grads[li] = (dW, db)
        dY = dX
    return loss, grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns the
    new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def flatten(params):
    """Parameters as one array: W_0, b_0, W_1, b_1, ... (row-major W)."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(flat, sizes):
    params, off = [], 0
    for cin, cout in zip(sizes[:-1], sizes[1:]):
        W = flat[off:off + TAPS * cin * cout].reshape(TAPS * cin, cout)
        off += TAPS * cin * cout
        b = flat[off:off + cout]
        off += cout
        params.append((W, b))
    return params
