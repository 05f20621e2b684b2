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


def test_bf16_round_exact_binary_cases():
    # BF16 keeps 7 fraction bits: near 1 the grid is 1 + k 2^-7; halfway cases go to even k
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + e + 2.0 ** -20, -(1 + 3 * e), 3.0 * 2.0 ** -130,
                     65535.0, 0.0])
    ref = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -(1 + 2.0 ** -6), 3.0 * 2.0 ** -130,
                    65536.0, 0.0])
    assert np.array_equal(cnn.bf16_round(vals), ref)


def _identity_net():
    """Every stored value of this network is a small integer times a power of
    two: BF16 storage must then change nothing."""
    params = []
    w = np.zeros((64, 1, 3, 3)); w[:, 0, 1, 1] = 1.0
    params.append((w, np.zeros(64)))
    for _ in range(8):
        w = np.zeros((64, 64, 3, 3))
        w[np.arange(64), np.arange(64), 1, 1] = 1.0
        params.append((w, np.zeros(64)))
    w = np.zeros((1, 64, 3, 3)); w[0, :, 1, 1] = 1.0 / 64
    params.append((w, np.zeros(1)))
    return params


def test_bf16_mode_rounds_only_where_values_are_stored():
    params = _identity_net()
    rng = np.random.default_rng(8)
    r = rng.integers(-8, 9, (8, 8)).astype(np.float64)
    clean = rng.integers(-8, 9, (8, 8)).astype(np.float64)
    f64, _ = cnn.forward(r, params)
    f16, _ = cnn.forward(r, params, bf16=True)
    assert np.array_equal(f64, np.maximum(r, 0)) and np.array_equal(f16, f64)
    l64, g64 = cnn.mse_loss_and_grads(r, clean, params)
    l16, g16 = cnn.mse_loss_and_grads(r, clean, params, bf16=True)
    assert l16 == l64
    for (a, b), (c, d) in zip(g64, g16):
        assert np.array_equal(a, c) and np.array_equal(b, d)
    # a generic network does differ, by about BF16's unit roundoff per layer
    params = cnn.init_params(3)
    r = rng.standard_normal((10, 10))
    f64, _ = cnn.forward(r, params)
    f16, _ = cnn.forward(r, params, bf16=True)
    rel = np.linalg.norm(f16 - f64) / np.linalg.norm(f64)
    assert 1e-4 < rel < 3e-2, rel
