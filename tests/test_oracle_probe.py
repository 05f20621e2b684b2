"""Pins of the counter-based Rademacher probe (Sec. 4.3, eq. MC_SURE)."""
import numpy as np

from oracle import probe


def test_splitmix64_published_values():
    # Reference outputs of SplitMix64 (Steele, Lea & Flood 2014) for the generator seeded at
    # 1234567: each output is the finaliser applied to the state after k additions of the
    # golden-gamma increment, i.e. splitmix64(1234567 + (k-1) * gamma).
    gamma = 0x9E3779B97F4A7C15
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    states = np.array([(1234567 + k * gamma) % 2 ** 64 for k in range(5)], dtype=np.uint64)
    with np.errstate(over="ignore"):
        out = probe.splitmix64(states)
    assert [int(v) for v in out] == ref


def test_rademacher_moments():
    b = probe.rademacher(42, 3, 1 << 16)
    assert set(np.unique(b)) == {-1.0, 1.0}
    assert abs(b.mean()) < 4 / np.sqrt(b.size)
    c = probe.rademacher(42, 4, 1 << 16)
    assert abs(np.mean(b * c)) < 4 / np.sqrt(b.size)          # E[b b'^T] = 0 off-diagonal
    assert not np.array_equal(b, c)
    assert np.array_equal(b, probe.rademacher(42, 3, 1 << 16))   # counter-based: reproducible
