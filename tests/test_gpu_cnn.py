"""Residual CNN denoiser on MFMA against the FP64 oracle (same BF16-rounded weights).

Two oracle references:
  * the oracle in BF16-storage mode, which rounds to BF16 exactly where the
    kernels store BF16 (hidden activations, their tangents, the masked
    back-propagated gradients) and computes in FP64 otherwise;
  * the plain FP64 oracle.
The GPU differs from the BF16-mode oracle only in FP32 accumulation order,
but that does not keep two BF16 pipelines close: a stored value within an
FP32 rounding of a BF16 rounding boundary rounds the other way, each such
flip changes the next layer's sums over a 3x3x64 window, more values then
cross boundaries, and layer by layer the two pipelines drift apart to a
distance of the order of BF16's own rounding, the same order as either's
distance from FP64 (and the first layer's weight gradient, a sum over
pixels that cancels to a small fraction of its terms, magnifies both
alike).  So, with d16 = the BF16-mode oracle's distance from FP64 (what BF16
storage itself costs), every compared quantity must satisfy:
cosine with the BF16-mode oracle >= 0.999, distance from it <= 2 d16, and
distance from FP64 <= 3 d16 (plus a floor of 1e-4 relative).  A kernel error
larger than BF16 storage itself fails these.
"""
import math

import numpy as np
import pytest
import torch

from oracle import cnn as ocnn
from oracle.probe import rademacher
from paper_1609_04661_amd import synth

pytestmark = pytest.mark.gpu


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def oracle_params(net):
    return [(bf16_round(w), b) for w, b in net.layers()]


def cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def check_vs_oracles(got, ref16, ref64, what):
    """got against the BF16-storage oracle and the FP64 oracle, in units of
    the distance BF16 storage itself puts between the two oracles."""
    d16 = rel(ref16, ref64)
    c = cos(got, ref16)
    r16, r64 = rel(got, ref16), rel(got, ref64)
    print(what, "cos %.6f  rel16 %.2e  rel64 %.2e  d16 %.2e" % (c, r16, r64, d16))
    assert c >= 0.999 and r16 <= 2.0 * d16 + 1e-4 and r64 <= 3.0 * d16 + 1e-4, \
        (what, c, r16, r64, d16)


def test_cnn_forward_matches_oracle(gpu_lib):
    net = gpu_lib.CnnNet(seed=3)
    params = oracle_params(net)
    rng = np.random.default_rng(0)
    imgs = rng.standard_normal((2, 40, 36))
    out = net.forward(torch.as_tensor(imgs, dtype=torch.float32).cuda())
    torch.cuda.synchronize()
    out = out.cpu().double().numpy()
    for k in range(2):
        r = imgs[k].astype(np.float32).astype(np.float64)
        f64, _ = ocnn.forward(r, params)
        f16, _ = ocnn.forward(r, params, bf16=True)
        f_gpu = r - out[k]
        check_vs_oracles(f_gpu, f16, f64, "f")


def test_cnn_gradients_match_oracle(gpu_lib):
    net = gpu_lib.CnnNet(seed=5)
    params = oracle_params(net)
    rng = np.random.default_rng(1)
    clean = rng.standard_normal((2, 24, 20)).astype(np.float32).astype(np.float64)
    noisy = (clean + 0.3 * rng.standard_normal((2, 24, 20))).astype(np.float32).astype(np.float64)
    loss = net.train_step(torch.as_tensor(noisy, dtype=torch.float32).cuda(),
                          torch.as_tensor(clean, dtype=torch.float32).cuda(), lr=1e-30)
    torch.cuda.synchronize()
    g_gpu = net.grad.cpu().double().numpy()
    refs = {}
    for bf in (False, True):
        ref_loss, ref_grads = 0.0, None
        for k in range(2):
            l, g = ocnn.mse_loss_and_grads(noisy[k], clean[k], params, bf16=bf)
            ref_loss += 0.5 * l
            g = [(0.5 * dw, 0.5 * db) for dw, db in g]
            ref_grads = g if ref_grads is None else [(a + c, b + d) for (a, b), (c, d) in zip(ref_grads, g)]
        refs[bf] = (ref_loss, ref_grads)
    assert abs(float(loss.item()) - refs[True][0]) <= 1e-4 * refs[True][0]
    off = 0
    stats = []
    for l, ((dw64, db64), (dw16, db16)) in enumerate(zip(refs[False][1], refs[True][1])):
        gw = g_gpu[off:off + dw64.size].reshape(dw64.shape)
        gb = g_gpu[off + dw64.size:off + dw64.size + db64.size]
        off += dw64.size + db64.size
        stats.append((l, round(cos(gw, dw16), 6), round(rel(gw, dw16), 5), round(rel(gw, dw64), 4),
                      round(rel(dw16, dw64), 4)))
        check_vs_oracles(gw, dw16, dw64, ("dW", l))
        check_vs_oracles(gb, db16, db64, ("db", l))
    print(stats)


@pytest.mark.parametrize("I", [48, 70, 288])
def test_cnn_denoise_and_tangent_divergence(gpu_lib, I):
    """The fused forward + tangent passes of the denoiser (a ragged tile tail
    at 70; at 288, 324 tiles of 16 x 16, more than the 256 workgroups a layer
    launches, so every workgroup walks several tiles): D(r) bitwise equal to
    the forward-only kernels, f and the tangent divergence against the
    oracle."""
    g = synth.geometry(synth.PARALLEL, I, 1.0, 4, I + 1, math.pi)
    plan = gpu_lib.Plan(g)
    net = gpu_lib.CnnNet(seed=7)
    params = oracle_params(net)
    r = np.random.default_rng(2).standard_normal((I, I)).astype(np.float32).astype(np.float64)
    p = gpu_lib.make_params(gpu_lib.DEN_CNN, net=net, n_pixels=I * I)
    x, div = gpu_lib.denoise(plan, gpu_lib.DEN_CNN, p, torch.as_tensor(r, dtype=torch.float32).cuda(),
                             torch.ones(1, dtype=torch.float64, device="cuda"), probe_seed=11,
                             iteration=2)
    torch.cuda.synchronize()
    x_fwd = net.forward(torch.as_tensor(r, dtype=torch.float32).cuda()[None])[0]
    torch.cuda.synchronize()
    assert torch.equal(x, x_fwd.reshape(x.shape))
    f64, _ = ocnn.forward(r, params)
    f16, _ = ocnn.forward(r, params, bf16=True)
    f_gpu = r - x.cpu().double().numpy()
    check_vs_oracles(f_gpu, f16, f64, "f")
    b = rademacher(11, 2, I * I).reshape(I, I)
    d16 = ocnn.tangent_divergence(r, params, b, bf16=True)
    d64 = ocnn.tangent_divergence(r, params, b)
    got = float(div.item())
    # 1 - div = b^T J_f b / N is the part the network contributes
    floor = 1e-4 * abs(1.0 - d64)
    print("tangent div gpu %.6f bf16-oracle %.6f fp64-oracle %.6f" % (got, d16, d64))
    assert abs(got - d16) <= 2.0 * abs(d16 - d64) + floor, (got, d16, d64)
    assert abs(got - d64) <= 3.0 * abs(d16 - d64) + floor, (got, d16, d64)


def test_cnn_training_reduces_loss(gpu_lib):
    net = gpu_lib.CnnNet(seed=9)
    rng = np.random.default_rng(3)
    yy, xx = np.mgrid[0:32, 0:32]
    clean = np.stack([np.sin(xx / (3 + k)) * np.cos(yy / (4 + k)) for k in range(4)])
    noisy = clean + 0.2 * rng.standard_normal(clean.shape)
    n_t = torch.as_tensor(noisy, dtype=torch.float32).cuda()
    c_t = torch.as_tensor(clean, dtype=torch.float32).cuda()
    losses = [float(net.train_step(n_t, c_t, lr=1e-3).item()) for _ in range(60)]
    assert losses[-1] < 0.5 * losses[0], losses[::10]
