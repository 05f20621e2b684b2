"""Write the stored oracle results that the full-size GPU parity tests compare with.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators
(``paper_1609_04661_amd.synth``, which hold none of the method's arithmetic).
Run from the repository root:

    python tests/golden/make_golden.py [c2] [c3] [c5]

Each case stores, in ``tests/golden/<case>.npz``:
  * the oracle's D-GAMP-CT result mu = V^-1 x^T (FP32 copy; for the
    1024 x 1024 case every second row and column, ``stride`` 2, to keep the
    file small) and its PSNR over the full image against the phantom
    (Sec. 6 reading: 10 log10(max(mu_true)^2 / MSE));
  * the per-iteration log (tau_p, tau_s, tau_r, div, tau_x) of Algorithm 1;
  * the scalar ||A V^-1||_F^2 the run used (Hutchinson, 16 probes, seed 99),
    so that the GPU run is handed the same number;
  * checksums of the counts y, so a test can confirm it rebuilt the same input;
  * the oracle's own sensitivity: the same run with every iterate x^{t+1}
    multiplied by (1 + delta xi), xi a seeded +-1 field per iteration and
    delta = 2e-5 (the denoiser's FP32 parity bound), and its distance from
    the unperturbed run (mu relative L2, PSNR difference).  The tests derive
    their full-run tolerance from it.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import _lib  # noqa: E402
from oracle import denoisers as oden  # noqa: E402
from oracle import gamp as ogamp  # noqa: E402
from oracle import metrics, radon  # noqa: E402
from paper_1609_04661_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
DELTA = 2e-5


def c3_slice():
    """The first 384 x 384 slice of the uneven batch (seed 1003)."""
    for s in synth.batch_slices(1003, 64):
        if s["geom"]["n"] == 384:
            return s
    raise RuntimeError("no 384 slice")


CASES = {
    # headline: 512^2, 64 parallel views x 729 bins, I0 1e5, NLM, 50 iterations, eta 0.15
    "c2": lambda: dict(geom=synth.c2_geometry(), mu=synth.ellipse_phantom(512, 1002),
                       i0=1e5, seed=1002, T=50, eta=0.15, probe_seed=7),
    # uneven batch slice at its configured 30 iterations
    "c3": lambda: (lambda s: dict(geom=s["geom"], mu=synth.ellipse_phantom(384, s["seed"]),
                                  i0=s["i0"], seed=s["seed"], T=30, eta=0.15,
                                  probe_seed=7))(c3_slice()),
    # fan-beam low-dose slice 0 (1024^2, 0.5 mm, 128 views over 360 deg, I0 5e3), 3 iterations
    "c5": lambda: (lambda s: dict(geom=s["geom"],
                                  mu=synth.ellipse_phantom(1024, s["seed"], pixel_mm=0.5,
                                                           inserts=s["inserts"]),
                                  i0=s["i0"], seed=s["seed"], T=3, eta=0.15,
                                  probe_seed=7, stride=2))(synth.c5_slices(1005, 16)[0]),
}


def run_case(name):
    c = CASES[name]()
    g, mu, T, eta = c["geom"], c["mu"], c["T"], c["eta"]
    R = radon.Radon(g)
    t0 = time.time()
    y = synth.poisson_counts(R.project(mu), c["i0"], c["seed"])
    fro2 = ogamp.fro2_hutchinson(R, 16, 99)
    kw = dict(eta_x=eta, eta_s=eta)
    mu_hat, log, clamps = ogamp.dgamp_ct(R, y, c["i0"], fro2, T, oden.NLM, {}, c["probe_seed"], **kw)
    t1 = time.time()

    def perturb(t, x, _):
        xi = 1.0 - 2.0 * np.random.default_rng(4242 + t).integers(0, 2, x.size)
        x *= 1.0 + DELTA * xi

    mu_p, _, _ = ogamp.dgamp_ct(R, y, c["i0"], fro2, T, oden.NLM, {}, c["probe_seed"],
                                callback=perturb, **kw)
    sens_rel = float(np.linalg.norm(mu_p - mu_hat) / np.linalg.norm(mu_hat))
    psnr = metrics.psnr(mu_hat, mu)
    sens_psnr = abs(metrics.psnr(mu_p, mu) - psnr)
    keys = ("tau_p", "tau_s", "tau_r", "div", "tau_x")
    L = np.array([[e[k] for k in keys] for e in log])
    stride = c.get("stride", 1)
    meta = dict(case=name, T=T, eta=eta, i0=c["i0"], seed=c["seed"], probe_seed=c["probe_seed"],
                stride=stride,
                fro2_probes=16, fro2_seed=99, geom=g, clamps=clamps, delta=DELTA,
                threads=_lib.set_threads(0), oracle_seconds=t1 - t0)
    _lib.set_threads(meta["threads"])
    np.savez_compressed(os.path.join(HERE, name + ".npz"),
                        mu_hat=mu_hat[::stride, ::stride].astype(np.float32),
                        log=L, fro2=np.float64(fro2), psnr=np.float64(psnr),
                        y_sum=np.float64(y.sum()), y_sq=np.float64((y * y).sum()),
                        sens_rel=np.float64(sens_rel), sens_psnr=np.float64(sens_psnr),
                        meta=np.array(json.dumps(meta)))
    print("%s: psnr %.4f dB, sensitivity rel %.3e / %.4f dB, clamps %d, oracle %.1f s"
          % (name, psnr, sens_rel, sens_psnr, clamps, t1 - t0), flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        run_case(name)
