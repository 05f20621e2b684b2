"""Benchmark: D-GAMP-CT iterations per second on one MI355X.

Workload (the configuration the headline metric is quoted on): 512 x 512
image (1 mm pixels), parallel beam, 64 views over 180 degrees, 729 bins,
Poisson counts at I0 = 1e5, patch-based (non-local means) denoiser with a
one-probe Monte-Carlo divergence.  Inputs are synthetic (seeded ellipse +
texture phantom, counts drawn from the library's own projection) and are
resident in HBM before timing starts.

One step = one full D-GAMP-CT iteration (V^-1 x, A, Poisson channel, A^T,
V^-1 g + r update, denoiser on r and r + eps b, divergence + tau_x).
The timed region runs `--steps` iterations from a fresh state through the C
ABI, bracketed by torch.cuda.synchronize(); HIP events recorded by the
library between the phases of every timed iteration give the per-phase
durations used for the roofline fields.

Prints one JSON line.  With `--gpus N`, N > 1 exits with a message: this
build runs on one GPU.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D-GAMP-CT iters/s & A+Aᵀ GB/s at 512², 64 views; learned vs plain at equal PSNR"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_TFLOPS = 157.3

# configured recursion for this workload (damping of means and variances)
CFG = dict(i0=1e5, seed=1002, probe_seed=7, eta=0.15, tau_x0=1.0, fro2_probes=16,
           nlm=dict(pr=2, sr=10, hfac=0.4))


def nlm_flops_per_pixel(pr, sr):
    """Algorithmic FP32 operations of the non-local-means kernel per output
    pixel: per search offset, one difference and one square per pixel of the
    (tile + patch halo) region (amortised 2), a separable box sum of
    2 (2 pr + 1) additions, and the weight: subtract, max, multiply, exp,
    weight sum, weighted accumulate (6)."""
    per_offset = 2 + 2 * (2 * pr + 1) + 6
    return (2 * sr + 1) ** 2 * per_offset


class HipEvents:
    """hipEvent_t handles through the HIP runtime torch already loaded."""

    def __init__(self, n):
        self.L = ctypes.CDLL("libamdhip64.so.7")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.L.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * n)()
        for k in range(n):
            h = ctypes.c_void_p()
            rc = self.L.hipEventCreate(ctypes.byref(h))
            if rc != 0:
                raise RuntimeError("hipEventCreate failed: %d" % rc)
            self.arr[k] = h
        self.n = n

    def ms(self, a, b):
        out = ctypes.c_float()
        rc = self.L.hipEventElapsedTime(ctypes.byref(out), self.arr[a], self.arr[b])
        if rc != 0:
            raise RuntimeError("hipEventElapsedTime failed: %d" % rc)
        return float(out.value)

    def close(self):
        for k in range(self.n):
            self.L.hipEventDestroy(self.arr[k])


def cpu_baseline(geom, mu, y, fro2, iters):
    """The FP64 oracle on the same inputs, `iters` iterations, host cores."""
    from oracle import denoisers as oden
    from oracle import gamp as ogamp
    from oracle import radon
    R = radon.Radon(geom)
    t0 = time.perf_counter()
    ogamp.dgamp_ct(R, y, CFG["i0"], fro2, iters, oden.NLM, dict(CFG["nlm"]),
                   CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    return dict(value=iters / dt, unit="iter/s", cores=cores, kind="oracle",
                sample="%d D-GAMP-CT iterations of the same 512x512 / 64-view workload "
                       "(FP64, C loops with OpenMP over %d threads, numpy FFTs), %.1f s"
                % (iters, cores, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the work would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1609_04661_amd import api, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    api.load()
    geom = synth.c2_geometry()
    plan = api.Plan(geom)
    I, N, M = plan.I, plan.N, plan.M
    mu = synth.ellipse_phantom(I, CFG["seed"])
    mu_d = torch.as_tensor(mu, dtype=torch.float32).cuda()
    z = api.ct_project(plan, mu_d)
    torch.cuda.synchronize()
    y = synth.poisson_counts(z.cpu().double().numpy(), CFG["i0"], CFG["seed"])
    y_d = torch.as_tensor(y, dtype=torch.float32).cuda()
    fro2 = float(api.dg_fro2_hutchinson(plan, CFG["fro2_probes"], 99).item())
    params = api.make_params(api.DEN_NLM, **CFG["nlm"])
    work = plan.workspace(api.OP_DGAMP)
    mu_out = torch.empty((I, I), dtype=torch.float32, device="cuda")

    def run(n, events=None, log=None):
        st = api.DgampState(plan, CFG["tau_x0"])
        api.dgamp_iterate(plan, y_d, st, n, fro2, CFG["i0"], api.DEN_NLM, params,
                          probe_seed=CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"],
                          mu_out=mu_out, log=log, work=work, phase_events=events)
        return st

    # warm-up (separate state)
    run(args.warmup)
    torch.cuda.synchronize()

    K = args.steps
    ev = HipEvents(K * (api.NPHASES + 1))
    log = torch.zeros(K * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = run(K, events=ev.arr, log=log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    status = float(st.scal[api.S_STATUS].item())

    phase_ms = {name: [] for name in api.PHASES}
    for it in range(K):
        base = it * (api.NPHASES + 1)
        for k, name in enumerate(api.PHASES):
            phase_ms[name].append(ev.ms(base + k, base + k + 1))
    ev.close()
    avg = {k: float(np.mean(v)) for k, v in phase_ms.items()}

    mu_hat = mu_out.cpu().double().numpy()
    with np.errstate(all="ignore"):
        mse = float(np.mean((mu_hat - mu) ** 2))
        psnr = 10 * math.log10(float(mu.max()) ** 2 / mse) if mse > 0 and math.isfinite(mse) else None

    nlm_flops = nlm_flops_per_pixel(CFG["nlm"]["pr"], CFG["nlm"]["sr"]) * N * 2  # r and r + eps b
    den_s = avg["denoise"] * 1e-3
    achieved_tflops = nlm_flops / den_s / 1e12
    a_bytes = 4.0 * (N + M)
    res = {
        "metric": METRIC,
        "value": K / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D-GAMP-CT 512x512, parallel 64 views x 729 bins, I0=1e5, "
                               "NLM 5x5/21x21 denoiser, MC divergence (1 Rademacher probe)",
                   "image": I, "views": geom["n_views"], "bins": geom["n_bins"],
                   "i0": CFG["i0"], "damping": CFG["eta"], "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "nlm_kernel",
                     "achieved": achieved_tflops, "peak": FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_TFLOPS,
                     "traffic": None},
        "phases_ms": avg,
        "A_GBps_algorithmic": a_bytes / (avg["project"] * 1e-3) / 1e9,
        "At_GBps_algorithmic": a_bytes / (avg["backproject"] * 1e-3) / 1e9,
        "A_At_frac_of_hbm_peak": (2 * a_bytes / ((avg["project"] + avg["backproject"]) * 1e-3) / 1e9)
        / HBM_PEAK_GBS,
        "psnr_db_after_steps": psnr,
        "nonfinite_pixels": int((~np.isfinite(mu_hat)).sum()),
        "final_log": dict(zip(api.LOG_FIELDS, [float(v) for v in
                                               log.view(K, api.LOG_STRIDE)[-1].cpu().numpy()])),
        "status": status,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(geom, mu, y, fro2, args.cpu_iters)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
