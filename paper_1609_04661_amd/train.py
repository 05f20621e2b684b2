"""Train the residual CNN denoiser with the library's own kernels.

Training pairs are (x + sigma psi, x) with x = V mu the preconditioned image
of a synthetic ellipse + texture phantom (the space the plug-in denoiser of
Sec. 4.3 works in), psi white Gaussian noise and sigma drawn log-uniformly
from the range of sqrt(tau_r) that plain D-GAMP-CT runs produce on the same
workload: the 512 x 512, 64-view, I0 = 1e5 run with the patch-based
denoiser (damping 0.15, 50 iterations; its per-iteration log is stored in
tests/golden/c2.npz, column tau_r) has sqrt(tau_r) from 2.47 at its first
iteration down to 0.027 at its 50th, and [0.02, 2.5] covers it.
Every forward, backward and Adam step runs in the HIP kernels
(dg_cnn_train_step); phantoms come from ``synth`` on host cores (a worker
pool forked before the GPU is touched, streamed in chunks) and are
preconditioned on the GPU (ct_precondition) as they arrive.

The shipped weights were made by

    python -m paper_1609_04661_amd.train --phantoms 20000 --steps 4000

(20000 phantoms from seed 1004 * 10^6 + k, batches of 16 random 128 x 128
crops with flips, Adam with cosine decay from 1e-3); the run's record is
weights/cnn_c2_x_space.json.
"""
import argparse
import json
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


def make_dataset(n_phantoms, side=512, procs=None, chunk=256):
    """x = V mu for every phantom, as a (n, side, side) CUDA tensor.  The
    phantoms are drawn on host cores by a worker pool that is forked before
    this process touches the GPU; chunks of them are preconditioned on the
    GPU as they arrive, so the host holds at most a chunk at a time."""
    procs = procs or min(16, os.cpu_count() or 1)
    jobs = [(side, TRAIN_SEED_BASE + k) for k in range(n_phantoms)]
    pool = mp.get_context("fork").Pool(procs)
    try:
        torch.cuda.set_device(0)
        api.load()
        g = synth.geometry(synth.PARALLEL, side, 1.0, 1, side + 1, math.pi)
        plan = api.Plan(g)
        work = plan.workspace(api.OP_PRECOND)
        xs = torch.empty((n_phantoms, side, side), dtype=torch.float32, device="cuda")
        for k, mu in enumerate(pool.imap(_phantom, jobs, chunksize=max(1, chunk // procs))):
            api.ct_precondition(plan, -1, torch.from_numpy(mu).cuda(), out=xs[k], work=work)
            if (k + 1) % 2000 == 0:
                print("phantoms %d / %d" % (k + 1, n_phantoms), flush=True)
        torch.cuda.synchronize()
    finally:
        pool.close()
        pool.join()
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


def train(n_phantoms=20000, steps=4000, batch=16, crop=128, lr=1e-3, sig_lo=0.02, sig_hi=2.5,
          seed=0, out=DEFAULT_WEIGHTS, log_every=100, init_scale=0.5):
    t0 = time.time()
    xs = make_dataset(n_phantoms)
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
        cmd = ("python -m paper_1609_04661_amd.train --phantoms %d --steps %d --batch %d --crop %d "
               "--lr %g --sig-lo %g --sig-hi %g --seed %d" % (n_phantoms, steps, batch, crop, lr,
                                                            sig_lo, sig_hi, seed))
        rec = dict(command=cmd,
                   phantoms=n_phantoms, phantom_seeds="%d + k" % TRAIN_SEED_BASE, steps=steps,
                   batch=batch, crop=crop, lr=lr, sigma_range=[sig_lo, sig_hi], seed=seed,
                   data_s=round(t_data, 1), train_s=round(t_train, 1),
                   loss_history=[(k, float("%.5g" % v)) for k, v in hist])
        with open(os.path.splitext(out)[0] + ".json", "w") as f:
            json.dump(rec, f, indent=1)
    return dict(net=net, history=hist, data_s=t_data, train_s=t_train)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--phantoms", type=int, default=20000)
    ap.add_argument("--steps", type=int, default=4000)
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
