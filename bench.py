"""Benchmark: D-GAMP-CT iterations per second on one MI355X.

Headline workload: 512 x 512 image (1 mm pixels), parallel beam, 64 views
over 180 degrees, 729 bins, Poisson counts at I0 = 1e5, patch-based
(non-local means) denoiser with a one-probe Monte-Carlo divergence.  Inputs
are synthetic (seeded ellipse + texture phantom, counts drawn from the
library's own projection) and are resident in HBM before timing starts.

One step = one full D-GAMP-CT iteration (V^-1 x, A, Poisson channel, A^T,
V^-1 g + r update, denoiser on r and r + eps b, divergence + tau_x).  The
timed region replays `--steps` iterations from a fresh state as one HIP
graph (dgamp_graph_create), bracketed by torch.cuda.synchronize(); `value`
is from the median of five replays.  The same iterations are also run with
eager launches, five times, with HIP events that the library records around
the denoiser of every iteration (on the stream the kernels run on): their
average is the dominant kernel's duration in the roofline fields (a graph
records no events), and an untimed eager rerun with every phase boundary
marked gives the per-phase durations.  Graph and eager runs compute the same
bits.

Further figures on the same line (each its own untimed-setup, timed-run pair):
  * learned_vs_plain: the residual CNN denoiser against NLM on the headline
    workload, PSNR after every iteration, time to reach the plain run's
    final PSNR;
  * batch_uneven: 64 independent slices (sides 256/384/512, 32/64/128 views,
    I0 log-uniform in [5e3, 1e5]) in one batch, 30 iterations, autotuned
    projector, HIP graph;
  * fan_lowdose: 16 fan-beam slices of 1024 x 1024 (0.5 mm) at I0 = 5e3,
    50 iterations of the batched learned-denoiser path in a HIP graph (and
    the NLM path beside it).

Prints one JSON line.  With `--gpus N`, N > 1 exits with a message: the
benchmark runs on one GPU only.
"""
import argparse
import ctypes
import json
import math
import multiprocessing as mp
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "D-GAMP-CT iters/s & A+Aᵀ GB/s at 512², 64 views; learned vs plain at equal PSNR"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0
WEIGHTS = os.path.join(ROOT, "paper_1609_04661_amd", "weights", "cnn_c2_x_space.safetensors")

# configured recursion for these workloads (damping of means and variances)
CFG = dict(i0=1e5, seed=1002, probe_seed=7, eta=0.15, tau_x0=1.0, fro2_probes=16,
           nlm=dict(pr=2, sr=10, hfac=0.4), tv=dict(alpha=1.0, iters=50),
           tvw=dict(iters=50, alphas={0: [0.02, 0.05, 0.1, 0.2], 1: [64.0, 256.0, 1024.0, 4096.0]},
                    fewer_steps=[10, 20]))
# HBM bytes per launch of nlm_kernel<2> at this workload, from two rocprofv3
# counter passes (FETCH_SIZE, WRITE_SIZE) scaled by a 256 MiB copy kernel
# (profiles/dgamp_c2_512x512_64views_hbm_traffic.md).  Set to None whenever
# that kernel changes until the counters are taken again.
NLM_TRAFFIC_BYTES = 7.250e6
# Counters of the two operators at this workload (per launch, rocprofv3 --pmc
# passes; profiles/radon_nlm_c2_512x512_64views_counters.md).  Set to None
# when either kernel changes until the counters are taken again.
A_AT_COUNTERS = {
    "A (project_kernel<8> + output channel)": {"us": 16.56, "valu_issue_frac": 0.70,
                                               "valu_instr_per_interaction": 21.8,
                                               "ta_busy_frac": 0.52},
    "At (backproject_kernel<0>)": {"us": 11.34, "valu_issue_frac": 0.87,
                                   "valu_instr_per_pixel_view": 23.2, "ta_busy_frac": 0.64}}
# dampings tried per denoiser for the time-to-equal-PSNR comparison (above
# 0.35 both recursions diverge on these inputs)
DAMPING_SWEEP = (0.15, 0.25, 0.35)
C3 = dict(seed=1003, slices=64, iters=30)
# timed runs of the headline (each K iterations from a fresh state); the
# reported value is the median
TIMED_RUNS = 5
C5 = dict(seed=1005, slices=16, iters=50)


def nlm_flops_per_pixel(pr, sr):
    """Algorithmic FP32 operations of non-local means per output pixel, as the
    cost model of the patch-based denoiser counts them: 12 per search offset
    (the squared difference and its separable box sum amortised over the
    patch, the weight and the two running sums), over (2 sr + 1)^2 offsets."""
    del pr
    return (2 * sr + 1) ** 2 * 12


def ray_pixel_interactions(geom):
    """Number of (ray, pixel) pairs with a non-zero chord: for every ray, the
    pixels a line crosses inside the I x I square, counted as its clipped
    length times (|cos| + |sin|) / h (one pixel per grid-line crossing) plus
    one.  Geometry only; this is the work count of one A or A^T."""
    import numpy as np
    I, h = geom["n"], geom["pixel_mm"]
    half = 0.5 * I * h
    nv, nb = geom["n_views"], geom["n_bins"]
    b = np.arange(nb) - 0.5 * (nb - 1)
    total = 0.0
    for k in range(nv):
        if geom["kind"] == 0:
            th = geom["angle0_rad"] + k * geom["span_rad"] / nv
            nx = np.full(nb, math.cos(th))
            ny = np.full(nb, math.sin(th))
            s = b * geom["bin_mm"]
        else:
            R = I * h / math.sqrt(2.0)
            dg = geom["dgamma_rad"] or 2.0 * math.asin(R / geom["dso_mm"]) / nb
            beta = geom["angle0_rad"] + k * geom["span_rad"] / nv
            ang = beta + b * dg + 0.5 * math.pi
            nx, ny = np.cos(ang), np.sin(ang)
            s = -geom["dso_mm"] * np.sin(b * dg)
        # clip the line {<u, n> = s} to the square: parametrise u = s n + t (-ny, nx)
        px, py, dx, dy = s * nx, s * ny, -ny, nx
        with np.errstate(divide="ignore", invalid="ignore"):
            tx0, tx1 = (-half - px) / dx, (half - px) / dx
            ty0, ty1 = (-half - py) / dy, (half - py) / dy
            lo = np.maximum(np.where(dx != 0, np.minimum(tx0, tx1), -np.inf),
                            np.where(dy != 0, np.minimum(ty0, ty1), -np.inf))
            hi = np.minimum(np.where(dx != 0, np.maximum(tx0, tx1), np.inf),
                            np.where(dy != 0, np.maximum(ty0, ty1), np.inf))
        inside = (np.abs(np.where(dx == 0, px, 0)) <= half) & (np.abs(np.where(dy == 0, py, 0)) <= half)
        ln = np.where(inside, np.maximum(hi - lo, 0.0), 0.0)
        total += float(np.sum(np.where(ln > 0, ln * (np.abs(nx) + np.abs(ny)) / h + 1.0, 0.0)))
    return total


def cnn_flops_per_pixel():
    """Multiply-adds x 2 of the 10-layer network per pixel: 1->64, 8 x 64->64,
    64->1, 3 x 3 taps."""
    return 2 * 9 * (64 + 8 * 64 * 64 + 64)


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


def _phantom_job(a):
    from paper_1609_04661_amd import synth
    n, seed, pixel_mm, inserts = a
    return synth.ellipse_phantom(n, seed, pixel_mm=pixel_mm, inserts=inserts).astype("float32")


def _gpu_may_be_initialised():
    """True when a profiler's preloaded library may already have set up the
    GPU in this process (rocprofv3 --pmc does so before the program starts):
    then no worker may be forked."""
    pre = os.environ.get("LD_PRELOAD", "")
    return "rocprof" in pre or any(k.startswith("ROCPROF") for k in os.environ)


def make_phantoms(jobs):
    """Phantoms on host cores: in a worker pool forked before this process
    touches the GPU, or in this process when the GPU may already be set up.
    The pool is closed and joined, so its workers exit normally."""
    procs = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    if procs == 1 or _gpu_may_be_initialised():
        return [_phantom_job(a) for a in jobs]
    pool = mp.get_context("fork").Pool(procs)
    try:
        out = pool.map(_phantom_job, jobs)
    finally:
        pool.close()
        pool.join()
    return out


def cpu_baseline(geom, mu, y, fro2, iters):
    """The FP64 oracle on the same inputs: `iters` iterations on all host
    threads, and one iteration on one thread."""
    from oracle import _lib as olib
    from oracle import denoisers as oden
    from oracle import gamp as ogamp
    from oracle import radon
    R = radon.Radon(geom)

    def run(n):
        t0 = time.perf_counter()
        ogamp.dgamp_ct(R, y, CFG["i0"], fro2, n, oden.NLM, dict(CFG["nlm"]),
                       CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
        return time.perf_counter() - t0

    cores = olib.set_threads(0)  # query
    olib.set_threads(cores)
    dt = run(iters)
    olib.set_threads(1)
    dt1 = run(1)
    olib.set_threads(cores)
    return dict(value=iters / dt, unit="iter/s", cores=cores, kind="oracle",
                sample="%d D-GAMP-CT iterations of the same 512x512 / 64-view workload "
                       "(FP64, C loops with OpenMP over %d threads, numpy FFTs), %.1f s"
                % (iters, cores, dt),
                one_thread_iter_per_s=1.0 / dt1)


def sync_time(fn, reps):
    import torch
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return statistics.median(out)


def first_reaching(curve, target):
    for k, v in enumerate(curve):
        if v == v and v >= target:
            return k + 1
    return None


def headline(api, synth, args, mu, results):
    import numpy as np
    import torch
    geom = synth.c2_geometry()
    plan = api.Plan(geom)
    I, N, M = plan.I, plan.N, plan.M
    mu_d = torch.as_tensor(mu, dtype=torch.float32).cuda()
    z = api.ct_project(plan, mu_d)
    torch.cuda.synchronize()
    y = synth.poisson_counts(z.cpu().double().numpy(), CFG["i0"], CFG["seed"])
    y_d = torch.as_tensor(y, dtype=torch.float32).cuda()
    fro2 = float(api.dg_fro2_hutchinson(plan, CFG["fro2_probes"], 99).item())
    params = api.make_params(api.DEN_NLM, **CFG["nlm"])
    work = plan.workspace(api.OP_DGAMP)
    mu_out = torch.empty((I, I), dtype=torch.float32, device="cuda")
    kw = dict(probe_seed=CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
    # the library's autotuner picks the projector's march segmentation for
    # this geometry (untimed, before the warm-up)
    results["projector_variant"] = plan.autotune(mu_d, mu_d.t().contiguous(), reps=10)
    # and the patch-based denoiser's tile split (8 or 4 wavefronts), on the
    # preconditioned phantom plus noise of the run's first iterations
    r_tune = torch.empty_like(mu_d)
    api.ct_precondition(plan, -1, mu_d, out=r_tune)
    r_tune += 0.1 * torch.randn_like(r_tune)
    if args.nlm_variant == "auto":
        results["nlm_variant"] = plan.autotune_nlm(r_tune, params, reps=10)
    else:
        plan.nlm_variant = int(args.nlm_variant)
        results["nlm_variant"] = plan.nlm_variant

    def run(n, events=None, log=None, mask=0):
        st = api.DgampState(plan, CFG["tau_x0"])
        api.dgamp_iterate(plan, y_d, st, n, fro2, CFG["i0"], api.DEN_NLM, params, mu_out=mu_out,
                          log=log, work=work, phase_events=events, phase_mask=mask, **kw)
        return st

    K = args.steps
    den = api.PHASES.index("denoise")  # the denoiser runs between marks den and den + 1
    den_mask = (1 << den) | (1 << (den + 1))
    wev = HipEvents(max(args.warmup, 1) * (api.NPHASES + 1))
    wlog = torch.zeros(max(args.warmup, 1) * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
    run(args.warmup, events=wev.arr, log=wlog, mask=den_mask)
    torch.cuda.synchronize()
    wev.close()

    # timed: RUNS runs of K iterations from a fresh state each; HIP events on
    # the library's stream bracket the denoiser (the dominant kernel) in every
    # timed iteration; `value` is from the median run
    ev = HipEvents(K * (api.NPHASES + 1))
    log = torch.zeros(K * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
    elapsed_runs, den_ms = [], []
    for _ in range(TIMED_RUNS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = run(K, events=ev.arr, mask=den_mask)
        torch.cuda.synchronize()
        elapsed_runs.append(time.perf_counter() - t0)
        den_ms += [ev.ms(it * (api.NPHASES + 1) + den, it * (api.NPHASES + 1) + den + 1)
                   for it in range(K)]
    elapsed = statistics.median(elapsed_runs)
    status = float(st.scal[api.S_STATUS].item())
    # untimed: the same iterations with every phase boundary marked and the
    # per-iteration scalars logged (the log's copy kernel stays out of the
    # timed runs)
    phase_ms = {name: [] for name in api.PHASES}
    run(K, events=ev.arr, log=log)
    torch.cuda.synchronize()
    for it in range(K):
        base = it * (api.NPHASES + 1)
        for k, name in enumerate(api.PHASES):
            phase_ms[name].append(ev.ms(base + k, base + k + 1))
    ev.close()
    avg = {k: float(np.mean(v)) for k, v in phase_ms.items()}
    nlm_ms = float(np.mean(den_ms))
    # mu_out now holds the rerun's result, identical to the timed run's (same
    # inputs, same probes, deterministic kernels)
    mu_hat = mu_out.cpu().double().numpy()
    psnr = float(api.dg_psnr(mu_out, mu_d).item())

    # timed: the same K iterations replayed from a graph (state reset
    # included), TIMED_RUNS replays; `value` is from the median
    gst = api.DgampState(plan, CFG["tau_x0"])
    G = api.DgampGraph(plan, y_d, gst, K, fro2, CFG["i0"], api.DEN_NLM, params,
                       tau_x0=CFG["tau_x0"], mu_out=mu_out, work=work, **kw)
    G.launch()
    graph_runs = []
    for _ in range(TIMED_RUNS):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.launch()
        torch.cuda.synchronize()
        graph_runs.append(time.perf_counter() - t0)
    graph_s = statistics.median(graph_runs)
    graph_psnr = float(api.dg_psnr(mu_out, mu_d).item())

    nlm_flops = nlm_flops_per_pixel(CFG["nlm"]["pr"], CFG["nlm"]["sr"]) * N * 2  # r, r + eps b
    achieved_tflops = nlm_flops / (nlm_ms * 1e-3) / 1e12
    a_bytes = 4.0 * (N + M)
    nnz = ray_pixel_interactions(geom)
    results.update({
        "value": K / graph_s,
        "ms_per_step": 1e3 * graph_s / K,
        "timed_runs_iter_per_s": [K / e for e in graph_runs],
        "eager_iter_per_s": K / elapsed,
        "eager_timed_runs_iter_per_s": [K / e for e in elapsed_runs],
        "roofline": {"bound": "alu",
                     "kernel": "nlm_kernel<2, %d>" % (4 if results["nlm_variant"] == 1 else 8),
                     "kernel_ms": nlm_ms,
                     "achieved": achieved_tflops, "peak": FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_TFLOPS,
                     "traffic": NLM_TRAFFIC_BYTES,
                     "traffic_algorithmic": 4.0 * 5 * N},
        "graph_ms_per_step": 1e3 * graph_s / K,
        "graph_iter_per_s": K / graph_s,
        "phases_ms": avg,
        "A_GBps_algorithmic": a_bytes / (avg["project"] * 1e-3) / 1e9,
        "At_GBps_algorithmic": a_bytes / (avg["backproject"] * 1e-3) / 1e9,
        "A_At_frac_of_hbm_peak": (2 * a_bytes / ((avg["project"] + avg["backproject"]) * 1e-3)
                                  / 1e9) / HBM_PEAK_GBS,
        "ray_pixel_interactions": nnz,
        "A_interactions_per_s": nnz / (avg["project"] * 1e-3),
        "At_interactions_per_s": nnz / (avg["backproject"] * 1e-3),
        "A_At_counters": A_AT_COUNTERS,
        "psnr_db_after_steps": psnr,
        "psnr_db_after_steps_graph": graph_psnr,
        "nonfinite_pixels": int((~np.isfinite(mu_hat)).sum()),
        "final_log": dict(zip(api.LOG_FIELDS, [float(v) for v in
                                               log.view(K, api.LOG_STRIDE)[-1].cpu().numpy()])),
        "status": status,
    })
    return dict(plan=plan, y=y, y_d=y_d, fro2=fro2, mu_d=mu_d, work=work, geom=geom, z_d=z)


def learned_vs_plain(api, args, h):
    """PSNR after every iteration for NLM and the CNN (same inputs, damping and
    probes); ms per iteration from graph replays of the whole run."""
    import torch
    plan, y_d, fro2, mu_d, work = h["plan"], h["y_d"], h["fro2"], h["mu_d"], h["work"]
    T = args.learned_iters
    net = api.CnnNet.load_file(WEIGHTS)
    kinds = {"plain_nlm": (api.DEN_NLM, api.make_params(api.DEN_NLM, **CFG["nlm"])),
             "learned_cnn": (api.DEN_CNN, api.make_params(api.DEN_CNN, net=net, n_pixels=plan.N))}
    kw = dict(probe_seed=CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
    out, curves = {}, {}
    mu_out = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    for name, (kind, params) in kinds.items():
        st = api.DgampState(plan, CFG["tau_x0"])
        ps = torch.empty(T, dtype=torch.float64, device="cuda")
        for t in range(T):
            api.dgamp_iterate(plan, y_d, st, 1, fro2, CFG["i0"], kind, params, mu_out=mu_out,
                              work=work, **kw)
            api.dg_psnr(mu_out, mu_d, out=ps[t:t + 1])
        curves[name] = [float(v) for v in ps.cpu().numpy()]
        gst = api.DgampState(plan, CFG["tau_x0"])
        G = api.DgampGraph(plan, y_d, gst, T, fro2, CFG["i0"], kind, params, tau_x0=CFG["tau_x0"],
                           mu_out=mu_out, work=work, **kw)
        G.launch()
        s = sync_time(G.launch, args.reps)
        c = curves[name]
        out[name] = dict(ms_per_iter=1e3 * s / T, iter_per_s=T / s, psnr_final=c[-1],
                         psnr_best=max(v for v in c if v == v),
                         psnr_every_5=[round(v, 3) for v in c[4::5]],
                         status=float(gst.scal[api.S_STATUS].item()))
    target = out["plain_nlm"]["psnr_final"]
    k_l = first_reaching(curves["learned_cnn"], target)
    t_plain = T * out["plain_nlm"]["ms_per_iter"]
    res = dict(iterations=T, damping=CFG["eta"], target_psnr_db=target, plain=out["plain_nlm"],
               learned=out["learned_cnn"], learned_iters_to_target=k_l,
               plain_ms_to_target=t_plain)
    if k_l is not None:
        t_l = k_l * out["learned_cnn"]["ms_per_iter"]
        res["learned_ms_to_target"] = t_l
        res["time_to_equal_psnr_speedup"] = t_plain / t_l
    res["raw_iter_rate_ratio"] = out["learned_cnn"]["iter_per_s"] / out["plain_nlm"]["iter_per_s"]
    res["cnn_tflops_per_iter"] = 2 * cnn_flops_per_pixel() * plan.N / 1e12

    # the damping is a tuning parameter of the recursion: each denoiser at the
    # damping (from DAMPING_SWEEP) that reaches the same target PSNR soonest;
    # ms per iteration does not depend on the damping
    own = {"etas_tried": list(DAMPING_SWEEP)}
    for name, (kind, params) in kinds.items():
        best = None
        for eta in DAMPING_SWEEP:
            st = api.DgampState(plan, CFG["tau_x0"])
            ps = torch.empty(T, dtype=torch.float64, device="cuda")
            for t in range(T):
                api.dgamp_iterate(plan, y_d, st, 1, fro2, CFG["i0"], kind, params,
                                  mu_out=mu_out, work=work, probe_seed=CFG["probe_seed"],
                                  eta_x=eta, eta_s=eta)
                api.dg_psnr(mu_out, mu_d, out=ps[t:t + 1])
            c = [float(v) for v in ps.cpu().numpy()]
            k = first_reaching(c, target)
            if k is not None and (best is None or k < best["iters_to_target"]):
                best = dict(eta=eta, iters_to_target=k, psnr_final=c[-1],
                            ms_to_target=k * out[name]["ms_per_iter"])
        own[name] = best
    if own["plain_nlm"] and own["learned_cnn"]:
        own["time_to_equal_psnr_speedup"] = (own["plain_nlm"]["ms_to_target"]
                                             / own["learned_cnn"]["ms_to_target"])
    res["own_damping"] = own
    return res


def ablation(api, h, T=50):
    """Sec. 7 style variants on the headline inputs (NLM): the Onsager term
    off, the damping the paper's toolbox runs used (eta_s 0.95, eta_x 0.65),
    and Algorithm 1 undamped, beside the configured run.  For each: the final
    PSNR, and how the variance the recursion predicts for x (tau_x) compares
    with the actual error of x against x_true = V mu (state-evolution check),
    as 10 log10(tau_x / MSE_x) averaged over iterations 5..T-1."""
    import numpy as np
    import torch
    plan, y_d, fro2, mu_d, work = h["plan"], h["y_d"], h["fro2"], h["mu_d"], h["work"]
    params = api.make_params(api.DEN_NLM, **CFG["nlm"])
    x_true = torch.empty_like(mu_d)
    api.ct_precondition(plan, -1, mu_d, out=x_true, work=plan.workspace(api.OP_PRECOND))
    peak = max(float(x_true.max().item()), 0.0)
    variants = {"configured": dict(eta_x=CFG["eta"], eta_s=CFG["eta"], onsager=True),
                "no_onsager": dict(eta_x=CFG["eta"], eta_s=CFG["eta"], onsager=False),
                "toolbox_damping": dict(eta_x=0.65, eta_s=0.95, onsager=True),
                "undamped": dict(eta_x=1.0, eta_s=1.0, onsager=True)}
    out = {}
    mu_out = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    for name, v in variants.items():
        st = api.DgampState(plan, CFG["tau_x0"])
        log = torch.zeros(T * api.LOG_STRIDE, dtype=torch.float64, device="cuda")
        px = torch.empty(T, dtype=torch.float64, device="cuda")
        for t in range(T):
            api.dgamp_iterate(plan, y_d, st, 1, fro2, CFG["i0"], api.DEN_NLM, params,
                              probe_seed=CFG["probe_seed"], eps_rel=1e-3,
                              log=log[t * api.LOG_STRIDE:(t + 1) * api.LOG_STRIDE],
                              mu_out=mu_out if t == T - 1 else None, work=work, **v)
            api.dg_psnr(st.x, x_true, out=px[t:t + 1])
        psnr_mu = float(api.dg_psnr(mu_out, mu_d).item())
        L = log.view(T, api.LOG_STRIDE).cpu().numpy()
        px = px.cpu().numpy()
        with np.errstate(all="ignore"):
            mse_x = peak * peak / np.power(10.0, px / 10.0)
            gap = 10.0 * np.log10(L[:, api.LOG_TAU_X] / mse_x)
        ok = np.isfinite(gap[5:])
        out[name] = dict(psnr_db=psnr_mu, status=float(st.scal[api.S_STATUS].item()),
                         se_gap_db_mean=float(np.mean(gap[5:][ok])) if ok.any() else None,
                         se_gap_db_last=float(gap[-1]) if np.isfinite(gap[-1]) else None)
        out[name]["_mse_x"] = mse_x
        out[name]["_tau_r"] = L[:, api.LOG_TAU_R]
    out["state_evolution"] = state_evolution(api, h, x_true, out, T)
    for v in out.values():
        v.pop("_mse_x", None)
        v.pop("_tau_r", None)
    return out


def state_evolution(api, h, x_true, runs, T):
    """The scalar state evolution (Sec. 4.4, eqs. SEasym / SE_matches, E_in,
    A_in) on the headline phantom, run by the library's dgamp_state_evolution
    with seeded standard-normal fields, beside the actual runs: the SE's
    predicted noise level of r (xi_r = tau_r) and predicted MSE of the
    denoiser's output E_in, against the actual run's tau_r and the actual MSE
    of its iterate x^{t+1} (with damping the iterate mixes D(r^t) with x^t,
    so the two MSEs differ in meaning; undamped they are the same quantity)."""
    import numpy as np
    import torch
    plan, y_d, fro2 = h["plan"], h["y_d"], h["fro2"]
    rng = np.random.default_rng(2024)
    n = torch.as_tensor(rng.standard_normal(plan.M), dtype=torch.float32).cuda()
    v = torch.as_tensor(rng.standard_normal(plan.N), dtype=torch.float32).cuda()
    params = api.make_params(api.DEN_NLM, **CFG["nlm"])
    z = h["z_d"].reshape(-1).contiguous()
    out = {}
    for name, eta in (("configured", CFG["eta"]), ("undamped", 1.0)):
        L = api.dgamp_state_evolution(plan, z, x_true.reshape(-1), y_d, n, v, T, fro2, CFG["i0"],
                                      api.DEN_NLM, params, probe_seed=CFG["probe_seed"],
                                      eta_x=eta, eta_s=eta)
        L = L.view(T, api.LOG_STRIDE).cpu().numpy()
        e_in, tau_r_se = L[:, api.SE_LOG_MSE], L[:, api.LOG_TAU_R]
        act = runs[name]
        with np.errstate(all="ignore"):
            gap = 10.0 * np.log10(e_in / act["_mse_x"])
            gap_r = 10.0 * np.log10(tau_r_se / act["_tau_r"])
        ok = np.isfinite(gap)
        out[name] = dict(eta=eta, se_status=float(L[-1, api.LOG_STATUS]),
                         se_mse_pred_every_5=[float("%.4g" % e) for e in e_in[4::5]],
                         actual_mse_x_every_5=[float("%.4g" % e) for e in act["_mse_x"][4::5]],
                         se_tau_r_every_5=[float("%.4g" % e) for e in tau_r_se[4::5]],
                         actual_tau_r_every_5=[float("%.4g" % e) for e in act["_tau_r"][4::5]],
                         mse_gap_db_mean=float(np.mean(gap[ok])) if ok.any() else None,
                         mse_gap_db_last=float(gap[-1]) if np.isfinite(gap[-1]) else None,
                         tau_r_gap_db_last=float(gap_r[-1]) if np.isfinite(gap_r[-1]) else None,
                         actual_valid_iterations=int(ok.sum()))
    return out


def prox_run(api, args, h, kind, params, T=50):
    """One plug-in run on the headline inputs at the configured damping: PSNR
    after every iteration, ms per iteration from a graph replay of the whole
    run, and the iteration at which it reaches the plain (NLM) run's final
    PSNR."""
    import torch
    plan, y_d, fro2, mu_d, work = h["plan"], h["y_d"], h["fro2"], h["mu_d"], h["work"]
    kw = dict(probe_seed=CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
    mu_out = torch.empty((plan.I, plan.I), dtype=torch.float32, device="cuda")
    st = api.DgampState(plan, CFG["tau_x0"])
    ps = torch.empty(T, dtype=torch.float64, device="cuda")
    for t in range(T):
        api.dgamp_iterate(plan, y_d, st, 1, fro2, CFG["i0"], kind, params, mu_out=mu_out,
                          work=work, **kw)
        api.dg_psnr(mu_out, mu_d, out=ps[t:t + 1])
    curve = [float(v) for v in ps.cpu().numpy()]
    gst = api.DgampState(plan, CFG["tau_x0"])
    G = api.DgampGraph(plan, y_d, gst, T, fro2, CFG["i0"], kind, params,
                       tau_x0=CFG["tau_x0"], mu_out=mu_out, work=work, **kw)
    G.launch()
    s = sync_time(G.launch, args.reps)
    out = dict(iterations=T, damping=CFG["eta"], ms_per_iter=1e3 * s / T, iter_per_s=T / s,
               psnr_final=curve[-1], psnr_best=max(curve),
               psnr_every_5=[round(v, 3) for v in curve[4::5]],
               status=float(gst.scal[api.S_STATUS].item()))
    target = h.get("plain_psnr")
    if target is not None:
        k = first_reaching(curve, target)
        out["plain_target_psnr_db"] = target
        out["iters_to_plain_psnr"] = k
        if k is not None:
            out["ms_to_plain_psnr"] = k * out["ms_per_iter"]
    return out


def proxtv(api, args, h, T=50):
    """The proximal-TV plug-ins (NEXT rank 2, Sec. 6): the l2 map at its
    configured alpha, and the metric map in both readings of the paper's norm
    ((V^T V)^-1 as the text writes it, V^T V as its TV figure's subscript),
    each over a small alpha sweep (no alpha is given for either)."""
    plan = h["plan"]
    out = prox_run(api, args, h, api.DEN_TV, api.make_params(api.DEN_TV, n_pixels=plan.N, **CFG["tv"]), T)
    out.update(alpha=CFG["tv"]["alpha"], dual_steps=CFG["tv"]["iters"])
    variants = {}
    for metric, name in ((0, "inv_VtV"), (1, "VtV")):
        runs = []
        for a in CFG["tvw"]["alphas"][metric]:
            prm = api.make_params(api.DEN_TVW, side=plan.I, alpha=a, iters=CFG["tvw"]["iters"],
                                  metric=metric)
            r = prox_run(api, args, h, api.DEN_TVW, prm, T)
            r["alpha"] = a
            runs.append(r)
        best = max(runs, key=lambda r: r["psnr_final"] if r["psnr_final"] == r["psnr_final"] else -1e9)
        # fewer primal-dual steps per call at the best alpha (K is not given either)
        steps = []
        for K in CFG["tvw"]["fewer_steps"]:
            prm = api.make_params(api.DEN_TVW, side=plan.I, alpha=best["alpha"], iters=K, metric=metric)
            r = prox_run(api, args, h, api.DEN_TVW, prm, T)
            steps.append(dict(primal_dual_steps=K, psnr_final=r["psnr_final"], ms_per_iter=r["ms_per_iter"],
                              iters_to_plain_psnr=r.get("iters_to_plain_psnr"),
                              ms_to_plain_psnr=r.get("ms_to_plain_psnr"), status=r["status"]))
        variants[name] = dict(metric=metric, primal_dual_steps=CFG["tvw"]["iters"], best=best,
                              sweep=[dict(alpha=r["alpha"], psnr_final=r["psnr_final"],
                                          psnr_every_5=r["psnr_every_5"], ms_per_iter=r["ms_per_iter"],
                                          status=r["status"]) for r in runs],
                              fewer_steps_at_best_alpha=steps)
    out["metric_variants"] = variants
    return out


def paper_ops(api, synth, h, plain_psnr, T=50):
    """The paper's own plug-in denoiser and its Fourier-slice operator.

    * BM3D-D-GAMP-CT on the headline inputs (same counts, damping, probes),
      time per iteration and PSNR beside the patch-based denoiser's run, and
      one BM3D call with its Monte-Carlo divergence (two denoiser passes).
    * The same method at the shape of the paper's own experiment (Sec. 6.1:
      a 512 x 512 slice, fan beam, 102 of 1024 views over 360 degrees,
      I0 = 1e5, about 10 iterations), on a synthetic phantom: seconds per
      iteration beside the paper's CPU figure (context, not a target).
    * The Fourier-slice operator pair (Sec. 2.4, eq. Radon_op) at the
      headline geometry: time per call beside the ray-driven pair, and the
      relative difference of the two models' projections of the phantom."""
    import numpy as np
    import torch
    out = {}
    plan, y_d, fro2, mu_d, work = h["plan"], h["y_d"], h["fro2"], h["mu_d"], h["work"]
    I = plan.I
    bm = api.make_params(api.DEN_BM3D, side=I)
    mu_out = torch.empty((I, I), dtype=torch.float32, device="cuda")
    ps = torch.empty(1, dtype=torch.float64, device="cuda")

    def run(n):
        st = api.DgampState(plan, CFG["tau_x0"])
        api.dgamp_iterate(plan, y_d, st, n, fro2, CFG["i0"], api.DEN_BM3D, bm, mu_out=mu_out,
                          work=work, probe_seed=CFG["probe_seed"], eta_x=CFG["eta"],
                          eta_s=CFG["eta"])
        return st
    run(2)
    s = sync_time(lambda: run(T), 3)
    st = run(T)
    api.dg_psnr(mu_out, mu_d, out=ps)
    r = torch.rand((I, I), device="cuda") * 0.3
    tau = torch.full((1,), 0.01, dtype=torch.float64, device="cuda")
    dwork = plan.workspace(api.OP_DENOISE)
    xo = torch.empty((I, I), dtype=torch.float32, device="cuda")
    dv = torch.empty(1, dtype=torch.float64, device="cuda")
    call = lambda: api.denoise(plan, api.DEN_BM3D, bm, r, tau, x_out=xo, div_out=dv, work=dwork)
    call()
    d_s = sync_time(call, 10)
    out["bm3d_c2"] = dict(iterations=T, ms_per_iter=1e3 * s / T, iter_per_s=T / s,
                          psnr_db=float(ps.item()), plain_patch_psnr_db=plain_psnr,
                          status=float(st.scal[api.S_STATUS].item()),
                          denoise_with_div_ms=1e3 * d_s,
                          megapixel_per_s_per_pass=2 * I * I / d_s / 1e6)
    # the paper's experiment shape
    g = synth.geometry(synth.FAN, 512, 0.7, 102, 736, 2 * np.pi, dso_mm=600.0, ddo_mm=500.0)
    P = api.Plan(g)
    mu = synth.ellipse_phantom(512, CFG["seed"] + 7, pixel_mm=0.7, inserts=0)
    m_d = torch.as_tensor(mu, dtype=torch.float32).cuda()
    z = api.ct_project(P, m_d)
    torch.cuda.synchronize()
    y = torch.as_tensor(synth.poisson_counts(z.cpu().double().numpy(), 1e5, CFG["seed"] + 7),
                        dtype=torch.float32).cuda()
    f2 = float(api.dg_fro2_hutchinson(P, CFG["fro2_probes"], 99).item())
    w2 = P.workspace(api.OP_DGAMP)
    o2 = torch.empty((512, 512), dtype=torch.float32, device="cuda")
    T2 = 50

    def run2(n, psnr_at=()):
        st2 = api.DgampState(P, CFG["tau_x0"])
        curve = {}
        done = 0
        for t in sorted(set(psnr_at) | {n}):
            api.dgamp_iterate(P, y, st2, t - done, f2, 1e5, api.DEN_BM3D, bm, mu_out=o2, work=w2,
                              probe_seed=CFG["probe_seed"], eta_x=CFG["eta"], eta_s=CFG["eta"])
            done = t
            if t in psnr_at:
                api.dg_psnr(o2, m_d, out=ps)
                curve[t] = float(ps.item())
        return st2, curve
    run2(2)
    s2 = sync_time(lambda: run2(T2), 3)
    st2, curve = run2(T2, psnr_at=(10, T2))
    out["bm3d_paper_shape"] = dict(geometry="fan 512x512 0.7 mm, 102 views over 360 deg, 736 bins, "
                                            "D_so 600 / D_od 500 mm, I0 1e5",
                                   iterations=T2, damping=CFG["eta"], s_per_iter=s2 / T2,
                                   psnr_db_at={str(k): v for k, v in curve.items()},
                                   status=float(st2.scal[api.S_STATUS].item()),
                                   paper_cpu_s_per_iter="18-27 (8-core Xeon, MATLAB + ASTRA)")
    # Fourier-slice operator
    F = api.FourierOp(h["geom"])
    zf = api.ct_project_fourier(F, mu_d)
    zr = api.ct_project(plan, mu_d)
    gf = api.ct_backproject_fourier(F, zf)
    a_f = sync_time(lambda: [api.ct_project_fourier(F, mu_d, zf) for _ in range(20)], 5) / 20
    at_f = sync_time(lambda: [api.ct_backproject_fourier(F, zf, gf) for _ in range(20)], 5) / 20
    mu_t = mu_d.t().contiguous()
    a_r = sync_time(lambda: [api.ct_project(plan, mu_d, mu_t, sino=zr) for _ in range(20)], 5) / 20
    gr = torch.empty_like(gf)
    at_r = sync_time(lambda: [api.ct_backproject(plan, zf, gr) for _ in range(20)], 5) / 20
    torch.cuda.synchronize()
    rel = float(torch.linalg.norm(zf - zr) / torch.linalg.norm(zr))
    out["fourier_c2"] = dict(A_us=1e6 * a_f, At_us=1e6 * at_f, ray_A_us=1e6 * a_r,
                             ray_At_us=1e6 * at_r, rel_diff_vs_ray_model=rel)
    return out


def operators(api, synth):
    """A and A^T on their own, per configured geometry: microseconds per call
    (median of 5 timings of 20 back-to-back calls after a warm-up, device
    inputs resident, projector segmentation tuned per plan) and ray-pixel
    interactions per second (ray_pixel_interactions)."""
    import torch
    geoms = {
        "C1 64^2 parallel, 30 views x 91": synth.c1_geometry(),
        "C2 512^2 parallel, 64 views x 729": synth.c2_geometry(),
        "C3 384^2 parallel, 96 views x 545": synth.geometry(synth.PARALLEL, 384, 1.0, 96, 545,
                                                             math.pi),
        "C5 1024^2 fan, 128 views x 1024": synth.c5_geometry(),
    }
    out = {}
    gen = torch.Generator(device="cuda").manual_seed(7)
    for name, g in geoms.items():
        P = api.Plan(g)
        mu = torch.rand((g["n"], g["n"]), device="cuda", generator=gen)
        mu_t = mu.t().contiguous()
        z = torch.rand((g["n_views"], g["n_bins"]), device="cuda", generator=gen)
        P.autotune(mu, mu_t, reps=10)
        zo = torch.empty_like(z)
        go = torch.empty_like(mu)
        for _ in range(3):
            api.ct_project(P, mu, mu_t, sino=zo)
            api.ct_backproject(P, z, go)
        a = sync_time(lambda: [api.ct_project(P, mu, mu_t, sino=zo) for _ in range(20)], 5) / 20
        at = sync_time(lambda: [api.ct_backproject(P, z, go) for _ in range(20)], 5) / 20
        nnz = ray_pixel_interactions(g)
        out[name] = dict(A_us=1e6 * a, At_us=1e6 * at, interactions=nnz,
                         A_interactions_per_s=nnz / a, At_interactions_per_s=nnz / at)
    return out


def run_batch(api, synth, slices, phantoms, den, T, reps, autotune, net=None):
    """One batch: counts from the library's projector, Hutchinson fro2 per
    slice, graph of the whole T-iteration run; returns timing and PSNRs."""
    import numpy as np
    import torch
    B = api.Batch([s["geom"] for s in slices])
    y_parts, fro2 = [], []
    cache = {}
    for s, mu in zip(slices, phantoms):
        key = tuple(sorted(s["geom"].items()))
        if key not in cache:
            P = api.Plan(s["geom"])
            cache[key] = (P, float(api.dg_fro2_hutchinson(P, CFG["fro2_probes"], 99).item()))
        P, f2 = cache[key]
        z = api.ct_project(P, torch.as_tensor(mu).cuda())
        torch.cuda.synchronize()
        y_parts.append(torch.as_tensor(synth.poisson_counts(z.cpu().double().numpy(), s["i0"],
                                                            s["seed"]), dtype=torch.float32)
                       .reshape(-1))
        fro2.append(f2)
    del cache
    y = torch.cat(y_parts).cuda()
    mu_true = torch.cat([torch.as_tensor(m).reshape(-1) for m in phantoms]).cuda()
    mu_out = torch.empty(B.totN, dtype=torch.float32, device="cuda")
    if den == "cnn":
        params = api.make_params(api.DEN_CNN, net=net, n_pixels=B.totN)
        kind = api.DEN_CNN
    else:
        params = api.make_params(api.DEN_NLM, **CFG["nlm"])
        kind = api.DEN_NLM
    B.bind(y, [s["i0"] for s in slices], fro2, kind, params, mu_out)
    variant = B.autotune(reps=5) if autotune else B.projector_variant
    G = B.graph(T, tau_x0=CFG["tau_x0"], probe_seed=CFG["probe_seed"], eta_x=CFG["eta"],
                eta_s=CFG["eta"])
    G.launch()
    s = sync_time(G.launch, reps)
    ps = torch.empty(B.n, dtype=torch.float64, device="cuda")
    for k in range(B.n):
        api.dg_psnr(B.image(mu_out, k), B.image(mu_true, k), out=ps[k:k + 1])
    ps = ps.cpu().numpy()
    status = B.scal.view(B.n, api.NSCAL)[:, api.S_STATUS].cpu().numpy()
    sides = [s["geom"]["n"] for s in slices]
    return dict(slices=B.n, iterations=T, ms_per_run=1e3 * s, ms_per_batch_iter=1e3 * s / T,
                slice_iter_per_s=B.n * T / s, pixels=int(B.totN), rays=int(B.totM),
                megapixel_iter_per_s=B.totN * T / s / 1e6, projector_variant=variant,
                nlm_variant=B.nlm_variant if den == "nlm" else None,
                sides_histogram={str(v): sides.count(v) for v in sorted(set(sides))},
                psnr_db_mean=float(np.nanmean(ps)), psnr_db_min=float(np.nanmin(ps)),
                slices_with_status=int((status != 0).sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=5, help="graph replays (median)")
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the learned, batched and fan-beam figures")
    ap.add_argument("--parts", default="headline,learned,batch,fan,ablation,paper_ops,operators",
                    help="comma-separated subset of headline,learned,batch,fan,ablation,paper_ops,"
                         "operators,proxtv (proxtv, the proximal-TV plug-ins with their alpha "
                         "sweeps, is opt-in)")
    ap.add_argument("--learned-iters", type=int, default=50)
    ap.add_argument("--nlm-variant", default="auto", choices=["auto", "0", "1"],
                    help="the headline's NLM tile split: tuned (auto) or fixed (0: 8 wavefronts, "
                         "1: 4), e.g. to take counters of one kernel")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device 3 times (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    parts = set(p.strip() for p in args.parts.split(",") if p.strip())
    if args.only_headline:
        parts = {"headline"}
    parts.add("headline")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    from paper_1609_04661_amd import synth
    c3 = synth.batch_slices(C3["seed"], C3["slices"])
    c5 = synth.c5_slices(C5["seed"], C5["slices"])
    jobs = [(512, CFG["seed"], 1.0, 0)]
    if "batch" in parts:
        jobs += [(s["geom"]["n"], s["seed"], 1.0, 0) for s in c3]
    if "fan" in parts:
        jobs += [(1024, s["seed"], 0.5, s["inserts"]) for s in c5]
    phantoms = make_phantoms(jobs)

    import numpy as np
    import torch

    from paper_1609_04661_amd import api
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    api.load()
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    res = {"metric": METRIC, "value": None, "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "D-GAMP-CT 512x512, parallel 64 views x 729 bins, I0=1e5, "
                                  "NLM 5x5/21x21 denoiser, MC divergence (1 Rademacher probe)",
                      "image": 512, "views": 64, "bins": 729, "i0": CFG["i0"],
                      "damping": CFG["eta"], "parallelism": "single GPU"}}
    mu = phantoms[0].astype(np.float64)
    h = headline(api, synth, args, mu, res)
    if "learned" in parts:
        print("learned vs plain", file=sys.stderr, flush=True)
        res["learned_vs_plain"] = learned_vs_plain(api, args, h)
    if "ablation" in parts:
        print("ablation", file=sys.stderr, flush=True)
        res["ablation"] = ablation(api, h)
    if "proxtv" in parts:
        print("proxtv", file=sys.stderr, flush=True)
        h["plain_psnr"] = res["psnr_db_after_steps"] if args.steps == 50 else None
        res["proxtv"] = proxtv(api, args, h)
    if "paper_ops" in parts:
        print("paper ops", file=sys.stderr, flush=True)
        res["paper_ops"] = paper_ops(api, synth, h, res.get("psnr_db_after_steps"))
    if "operators" in parts:
        print("operators", file=sys.stderr, flush=True)
        res["operators"] = operators(api, synth)
    if "batch" in parts:
        print("batch_uneven", file=sys.stderr, flush=True)
        res["batch_uneven"] = run_batch(api, synth, c3, phantoms[1:1 + len(c3)], "nlm",
                                        C3["iters"], args.reps, autotune=True)
    if "fan" in parts:
        print("fan_lowdose", file=sys.stderr, flush=True)
        net = api.CnnNet.load_file(WEIGHTS)
        p5 = phantoms[len(phantoms) - len(c5):]
        fan = run_batch(api, synth, c5, p5, "cnn", C5["iters"], max(1, args.reps // 2),
                        autotune=True, net=net)
        fan["cnn_tflops_achieved_upper"] = (2 * cnn_flops_per_pixel() * fan["pixels"]
                                            / (fan["ms_per_batch_iter"] * 1e-3) / 1e12)
        fan["plain_nlm"] = run_batch(api, synth, c5, p5, "nlm", C5["iters"], 1, autotune=True)
        res["fan_lowdose"] = fan
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(h["geom"], mu, h["y"], h["fro2"], args.cpu_iters)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
