"""Image-quality metrics, FP64 (test infrastructure).

Sec. 6 reports PSNR and SSIM.  Its PSNR sentence is garbled; the reading
used is PSNR = 10 log10(max(mu_true)^2 / MSE) with the MSE over all pixels.
SSIM follows Wang et al. 2004 (Gaussian window sigma 1.5, K1 = 0.01,
K2 = 0.03, data range max(mu_true)).

Parity: PSNR pinned by its definition on hand-computed cases.
"""
import math

import numpy as np


def psnr(est, ref):
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mse = float(np.mean((est - ref) ** 2))
    peak = float(np.max(ref))
    return 10.0 * math.log10(peak * peak / mse)


def ssim(est, ref):
    from scipy.ndimage import gaussian_filter
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    L = float(np.max(ref))
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    f = lambda a: gaussian_filter(a, 1.5, truncate=3.5)
    mx, my = f(est), f(ref)
    sxx = f(est * est) - mx * mx
    syy = f(ref * ref) - my * my
    sxy = f(est * ref) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(np.mean(s))
