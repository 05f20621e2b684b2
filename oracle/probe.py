"""Counter-based Rademacher probe for the Monte-Carlo divergence (test infrastructure).

Sec. 4.3 eq. MC_SURE estimates the divergence with one random probe vector b
(K = 1).  The paper draws b Gaussian; a +-1 (Rademacher) probe has the same
E[b b^T] = I, so the estimator stays unbiased.  b_i is drawn from a counter,
so that any implementation reproduces it without storing it:

    b_i = 1 - 2 * (SplitMix64(seed XOR (t << 32) XOR i) & 1)

where t is the GAMP iteration and SplitMix64 is the finaliser of Steele, Lea
& Flood (OOPSLA 2014): z += 0x9E3779B97F4A7C15;
z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) * 0x94D049BB133111EB;
return z ^ (z >> 31)   (all arithmetic mod 2^64).

Parity: pinned (published SplitMix64 output values; first and second moments).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output for state x (array of uint64); one step."""
    z = np.asarray(x, dtype=np.uint64) + _GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def rademacher(seed, t, n):
    """b in {-1, +1}^n for probe seed and iteration t, FP64."""
    with np.errstate(over="ignore"):
        key = np.uint64(seed) ^ (np.uint64(t) << np.uint64(32))
        i = np.arange(n, dtype=np.uint64)
        bits = splitmix64(key ^ i) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)
