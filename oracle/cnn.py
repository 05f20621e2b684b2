"""FP64 residual CNN denoiser: forward, backward and divergence (test infrastructure).

The learned plug-in denoiser (not in the paper, which mentions residual
CNN denoisers only as related work; the method treats D as a black box,
Sec. 4.3):  D(r) = r - f(r), where f is
    conv 1->64, ReLU, 8 x (conv 64->64, ReLU), conv 64->1,
every conv 3 x 3 with bias, zero padding, cross-correlation
    out[o, y, x] = b[o] + sum_{i, ty, tx} w[o, i, ty, tx] in[i, y + ty - 1, x + tx - 1].
Parameters are a list of (w, b) per layer with w of shape (co, ci, 3, 3).

The divergence follows eq. MC_SURE with the finite difference
b^T (D(r + eps b) - D(r)) / (N eps).

BF16 storage (``bf16=True``): the learned denoiser keeps its activations in
BF16 (the configured network: BF16 weights and activations, FP32
accumulation).  With ``bf16=True`` the oracle rounds, in FP64 otherwise,
at exactly the points where such a network stores BF16 values: every hidden
layer's post-ReLU activation (and its tangent) in the forward pass, and the
back-propagated gradient after each ReLU mask in the backward pass.  The
rounding is IEEE round-to-nearest-even to 8 significant bits of the FP32
value.  This separates the error BF16 storage itself causes (amplified
through cancelling sums over pixels in the weight gradients) from any
error of an implementation that stores BF16 at those points.

Parity: forward/backward pinned by central finite differences of the loss
and by linearity checks; bf16 rounding pinned by exact binary cases and by
the bf16 mode equalling the FP64 mode where every stored value is exactly
representable; against the paper unpinned (the paper has no CNN).
"""
import numpy as np

CHANNELS = 64
N_MID = 8


def shapes():
    s = [((CHANNELS, 1, 3, 3), (CHANNELS,))]
    s += [((CHANNELS, CHANNELS, 3, 3), (CHANNELS,))] * N_MID
    s += [((1, CHANNELS, 3, 3), (1,))]
    return s


def init_params(seed, scale=1.0):
    """He-style random initialisation (float64)."""
    rng = np.random.default_rng(seed)
    out = []
    for ws, bs in shapes():
        fan_in = ws[1] * 9
        w = rng.standard_normal(ws) * np.sqrt(2.0 / fan_in) * scale
        b = rng.standard_normal(bs) * 0.01
        out.append((w, b))
    return out


def conv3x3(x, w, b=None):
    """x: (ci, H, W) -> (co, H, W), zero padding."""
    ci, H, W = x.shape
    xp = np.zeros((ci, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], H, W))
    for ty in range(3):
        for tx in range(3):
            patch = xp[:, ty:ty + H, tx:tx + W].reshape(ci, -1)
            # (a contiguous copy of the tap's weight matrix keeps the product on
            # the library's fast path; the arithmetic is unchanged)
            out += (np.ascontiguousarray(w[:, :, ty, tx]) @ patch).reshape(-1, H, W)
    if b is not None:
        out += b[:, None, None]
    return out


def conv3x3_input_grad(g, w):
    """d(sum g * conv(x))/dx for g: (co, H, W) -> (ci, H, W)."""
    co, H, W = g.shape
    gp = np.zeros((co, H + 2, W + 2))
    gp[:, 1:-1, 1:-1] = g
    out = np.zeros((w.shape[1], H, W))
    for ty in range(3):
        for tx in range(3):
            # x[y', x'] feeds out[y' - ty + 1, x' - tx + 1]
            patch = gp[:, 2 - ty:2 - ty + H, 2 - tx:2 - tx + W].reshape(co, -1)
            out += (np.ascontiguousarray(w[:, :, ty, tx].T) @ patch).reshape(-1, H, W)
    return out


def conv3x3_weight_grad(g, x):
    """d(sum g * conv(x))/dw and /db."""
    ci, H, W = x.shape
    xp = np.zeros((ci, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((g.shape[0], ci, 3, 3))
    g2 = g.reshape(g.shape[0], -1)
    for ty in range(3):
        for tx in range(3):
            dw[:, :, ty, tx] = g2 @ xp[:, ty:ty + H, tx:tx + W].reshape(ci, -1).T
    return dw, g2.sum(axis=1)


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even) of the FP32 value of a;
    returned as float64."""
    a32 = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(r, params, bf16=False):
    """f(r) and the post-ReLU activations of every hidden layer (BF16-rounded
    when bf16)."""
    a = np.asarray(r, dtype=np.float64)[None]
    acts = [a]
    for l, (w, b) in enumerate(params):
        z = conv3x3(a, w, b)
        if l < len(params) - 1:
            a = np.maximum(z, 0.0)
            if bf16:
                a = bf16_round(a)
        else:
            a = z
        acts.append(a)
    return a[0], acts


def denoise(r, params):
    f, _ = forward(r, params)
    return np.asarray(r, dtype=np.float64) - f


def backward(acts, params, g_f, bf16=False):
    """Gradients of sum(g_f * f) w.r.t. every (w, b) and w.r.t. the input r
    (the masked gradient BF16-rounded at every hidden layer when bf16)."""
    g = np.asarray(g_f, dtype=np.float64)[None]
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        w, b = params[l]
        if l < len(params) - 1:
            g = g * (acts[l + 1] > 0)
            if bf16:
                g = bf16_round(g)
        grads[l] = conv3x3_weight_grad(g, acts[l])
        g = conv3x3_input_grad(g, w)
    return grads, g[0]


def mse_loss_and_grads(noisy, clean, params, bf16=False):
    """L = mean((D(noisy) - clean)^2) for one image; gradients w.r.t. params."""
    f, acts = forward(noisy, params, bf16)
    res = noisy - f - clean
    n = res.size
    loss = float(np.sum(res * res) / n)
    g_f = -2.0 * res / n
    grads, _ = backward(acts, params, g_f, bf16)
    return loss, grads


def fd_divergence(r, params, b, eps):
    """eq. MC_SURE: b^T (D(r + eps b) - D(r)) / (N eps)."""
    d0 = denoise(r, params)
    d1 = denoise(r + eps * b, params)
    return float(np.sum(b * (d1 - d0)) / (r.size * eps))


def tangent_divergence(r, params, b, bf16=False):
    """b^T J_D(r) b / N with the ReLU pattern of r (the eps -> 0 limit); with
    bf16 the activations and the tangent are BF16-rounded per hidden layer."""
    _, acts = forward(r, params, bf16)
    t = np.asarray(b, dtype=np.float64)[None]
    for l, (w, _) in enumerate(params):
        t = conv3x3(t, w)
        if l < len(params) - 1:
            t = t * (acts[l + 1] > 0)
            if bf16:
                t = bf16_round(t)
    return float(np.sum(b * (b - t[0])) / r.size)
