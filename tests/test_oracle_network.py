"""Pins of the FP64 reference network (warm-start predictor)."""
import numpy as np

from oracle import network as N


def test_conv1d_is_circular_correlation():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 11, 3))
    W = rng.standard_normal((5 * 3, 4))
    b = rng.standard_normal(4)
    out = N.conv1d(X, W, b)
    # direct definition with explicit modular indexing
    ref = np.zeros_like(out)
    for bb in range(2):
        for l in range(11):
            for co in range(4):
                s = b[co]
                for tap in range(5):
                    for ci in range(3):
                        s += W[tap * 3 + ci, co] * X[bb, (l + tap - 2) % 11, ci]
                ref[bb, l, co] = s
    assert np.max(np.abs(out - ref)) < 1e-13
    # FFT form of circular correlation per (ci, co)
    Lf = np.fft.fft(X, axis=1)
    k = np.zeros((11, 3, 4))
    for tap in range(5):
        k[(tap - 2) % 11] += W[tap * 3:(tap + 1) * 3]
    Kf = np.fft.fft(k, axis=0)
    viafft = np.real(np.fft.ifft(np.einsum("blc,lco->blo", Lf, np.conj(Kf)), axis=1)) + b
    assert np.max(np.abs(viafft - out)) < 1e-12


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = N.init_params([3, 8, 8, 1], seed=5)
    X = rng.standard_normal((2, 9, 3))
    T = rng.standard_normal((2, 9))
    loss, grads = N.loss_and_grads(params, X, T)
    eps = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp, _ = N.loss_and_grads(params, X, T)
                flat[idx] = old - eps
                lm, _ = N.loss_and_grads(params, X, T)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - gflat[idx]) < 1e-6 * (1 + abs(fd)), (li, idx, fd, gflat[idx])


def test_gelu_derivative():
    z = np.linspace(-4, 4, 101)
    fd = (N.gelu(z + 1e-6) - N.gelu(z - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - N.gelu_grad(z))) < 1e-8


def test_adam_first_step_is_signed_lr():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, -2e2])
    p, m, v = N.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=0, atol=1e-15)
    # a constant gradient keeps the step at lr (bias corrections cancel)
    for t in range(2, 6):
        p2, m, v = N.adam_step(p, g, m, v, t, lr=0.01, eps=0.0)
        assert np.allclose(p2 - p, -0.01 * np.sign(g), rtol=1e-12, atol=0)
        p = p2


def test_flatten_roundtrip():
    params = N.init_params([10, 16, 16, 1], seed=3)
    back = N.unflatten(N.flatten(params), [10, 16, 16, 1])
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)
