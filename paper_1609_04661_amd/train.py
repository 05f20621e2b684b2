"""Train the residual CNN denoiser with the library's own kernels.

Training pairs are (x + sigma psi, x) with x = V mu the preconditioned image
of a synthetic ellipse + texture phantom (the space the plug-in denoiser of
Sec. 4.3 works in), psi white Gaussian noise and sigma drawn log-uniformly
from the range of sqrt(tau_r) that plain D-GAMP-CT runs produce on the same
workload.  Every forward, backward and Adam step runs in the HIP kernels
(dg_cnn_train_step); phantoms come from ``synth`` on host cores and are
preconditioned on the GPU (ct_precondition).

    python -m paper_1609_04661_amd.train --phantoms 256 --steps 2000 --out weights.safetensors
"""
import argparse
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import torch

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1609_04661_amd import api, synth  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "cnn_c2_x_space.safetensors")
TRAIN_SEED_BASE = 1004 * 1000000


def _phantom(args):
    n, seed = args
    return synth.ellipse_phantom(n, seed).astype(np.float32)


def make_phantoms(n_phantoms, side=512, procs=None):
    """Phantoms on host cores.  Call before the process touches the GPU: the
    worker pool is forked, and a forked child must not inherit a live GPU
    context."""
    procs = procs or min(16, os.cpu_count() or 1)
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_phantom, [(side, TRAIN_SEED_BASE + k) for k in range(n_phantoms)])


def make_dataset(mus):
    """x = V mu for every phantom, as a (n, side, side) CUDA tensor."""
    n_phantoms, side = len(mus), mus[0].shape[0]
    g = synth.geometry(synth.PARALLEL, side, 1.0, 1, side + 1, math.pi)
    plan = api.Plan(g)
    work = plan.workspace(api.OP_PRECOND)
    xs = torch.empty((n_phantoms, side, side), dtype=torch.float32, device="cuda")
    for k, mu in enumerate(mus):
        api.ct_precondition(plan, -1, torch.from_numpy(mu).cuda(), out=xs[k], work=work)
    torch.cuda.synchronize()
    return xs


def sample_batch(xs, batch, crop, sig_lo, sig_hi, gen):
    n, H, W = xs.shape
    idx = torch.randint(0, n, (batch,), generator=gen)
    oy = torch.randint(0, H - crop + 1, (batch,), generator=gen)
    ox = torch.randint(0, W - crop + 1, (batch,), generator=gen)
    flips = torch.randint(0, 8, (batch,), generator=gen)
    clean = torch.empty((batch, crop, crop), dtype=torch.float32, device="cuda")
    for b in range(batch):
        c = xs[idx[b], oy[b]:oy[b] + crop, ox[b]:ox[b] + crop]
        f = int(flips[b])
        if f & 1:
            c = c.flip(0)
        if f & 2:
            c = c.flip(1)
        if f & 4:
            c = c.t()
        clean[b] = c
    u = torch.rand((batch, 1, 1), generator=gen)
    sig = torch.exp(math.log(sig_lo) + u * (math.log(sig_hi) - math.log(sig_lo))).cuda()
    noise = torch.randn((batch, crop, crop), generator=gen).cuda()
    noisy = (clean + sig * noise).contiguous()
    return noisy, clean


def train(n_phantoms=256, steps=2000, batch=16, crop=128, lr=1e-3, sig_lo=0.02, sig_hi=2.5,
          seed=0, out=DEFAULT_WEIGHTS, log_every=100, init_scale=0.5):
    t0 = time.time()
    mus = make_phantoms(n_phantoms)
    torch.cuda.set_device(0)
    api.load()
    xs = make_dataset(mus)
    del mus
    t_data = time.time() - t0
    net = api.CnnNet(master=api.CnnNet.init_master(seed, scale=init_scale))
    gen = torch.Generator().manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t1 = time.time()
    for k in range(steps):
        noisy, clean = sample_batch(xs, batch, crop, sig_lo, sig_hi, gen)
        lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))  # cosine decay
        net.train_step(noisy, clean, lr_k, loss_out=loss)
        if (k + 1) % log_every == 0 or k == 0:
            v = float(loss.item())
            hist.append((k + 1, v))
            print("step %d loss %.4e lr %.2e" % (k + 1, v, lr_k), flush=True)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        net.save(out)
    return dict(net=net, history=hist, data_s=t_data, train_s=t_train)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--phantoms", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--sig-lo", type=float, default=0.02)
    ap.add_argument("--sig-hi", type=float, default=2.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args()
    r = train(a.phantoms, a.steps, a.batch, a.crop, a.lr, a.sig_lo, a.sig_hi, a.seed, a.out)
    print("data %.1f s, training %.1f s (%d steps), final loss %.4e" %
          (r["data_s"], r["train_s"], a.steps, r["history"][-1][1]))


if __name__ == "__main__":
    main()
