"""Pins of the oracle's FP64 residual CNN (forward, backward, divergence)."""
import numpy as np
from scipy.signal import correlate2d

from oracle import cnn


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 9, 7))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    out = cnn.conv3x3(x, w, b)
    for o in range(2):
        ref = b[o] + sum(correlate2d(x[i], w[o, i], mode="same", boundary="fill") for i in range(3))
        assert np.max(np.abs(out[o] - ref)) < 1e-12


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    params = cnn.init_params(3)
    noisy = rng.standard_normal((6, 6))
    clean = rng.standard_normal((6, 6))
    loss, grads = cnn.mse_loss_and_grads(noisy, clean, params)
    h = 1e-6
    for l in (0, 4, 9):
        w, b = params[l]
        for idx in [tuple(rng.integers(0, s) for s in w.shape) for _ in range(4)]:
            wp = w.copy(); wp[idx] += h
            wm = w.copy(); wm[idx] -= h
            pp = list(params); pp[l] = (wp, b)
            pm = list(params); pm[l] = (wm, b)
            fd = (cnn.mse_loss_and_grads(noisy, clean, pp)[0] - cnn.mse_loss_and_grads(noisy, clean, pm)[0]) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        k = int(rng.integers(0, b.size))
        bp = b.copy(); bp[k] += h
        bm = b.copy(); bm[k] -= h
        pp = list(params); pp[l] = (w, bp)
        pm = list(params); pm[l] = (w, bm)
        fd = (cnn.mse_loss_and_grads(noisy, clean, pp)[0] - cnn.mse_loss_and_grads(noisy, clean, pm)[0]) / (2 * h)
        assert abs(fd - grads[l][1][k]) <= 1e-6 * max(1.0, abs(fd))


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(4)
    r = rng.standard_normal((5, 5))
    g_f = rng.standard_normal((5, 5))
    f, acts = cnn.forward(r, params)
    _, g_in = cnn.backward(acts, params, g_f)
    h = 1e-6
    for idx in [(0, 0), (2, 3), (4, 4)]:
        rp = r.copy(); rp[idx] += h
        rm = r.copy(); rm[idx] -= h
        fd = (np.sum(g_f * cnn.forward(rp, params)[0]) - np.sum(g_f * cnn.forward(rm, params)[0])) / (2 * h)
        assert abs(fd - g_in[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_tangent_divergence_is_the_small_eps_limit():
    rng = np.random.default_rng(5)
    params = cnn.init_params(6)
    r = rng.standard_normal((12, 12))
    b = np.where(rng.random((12, 12)) < 0.5, -1.0, 1.0)
    t = cnn.tangent_divergence(r, params, b)
    fd = cnn.fd_divergence(r, params, b, 1e-7)
    assert abs(t - fd) < 1e-6
    # a linear network (no ReLU active flips) has the exact trace; identity check:
    zero = [(np.zeros_like(w), np.zeros_like(bb)) for w, bb in params]
    assert abs(cnn.tangent_divergence(r, zero, b) - 1.0) < 1e-15
