"""Pins of the oracle's traditional ziggurat (Table 1, right column), the A/B
counterpart of the modified sampler: the stack constants against the
published values of Marsaglia & Tsang (J. Stat. Software 5(8), 2000: 256
layers, exponential r = 7.69711747013104972, v = 0.0039496598225815571993;
normal r = 3.6541528853610088, v = 0.00492867323399), the paper's 97.8 %
quick exit for the exponential (Table 1), equal layer areas in exact
arithmetic, and the output distribution."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import special, stats

from helpers import EXP, NORMAL

P_MIN = 1e-4


def test_published_constants(O):
    e = O.trad_arrays(EXP)
    n = O.trad_arrays(NORMAL)
    assert abs(e["r"] - 7.69711747013104972) < 1e-14 and abs(e["v"] - 0.0039496598225815571993) < 1e-17
    assert abs(n["r"] - 3.6541528853610088) < 1e-14 and abs(n["v"] - 0.00492867323399) < 1e-13


def test_quick_exit_rate(O):
    """Each layer is chosen with probability 1/n and quick-accepts a
    fraction k_i of its draws: 97.8 % for the exponential (Table 1)."""
    assert round(O.trad_arrays(EXP)["k"].mean(), 3) == 0.978
    assert 0.98 < O.trad_arrays(NORMAL)["k"].mean() < 0.99


@pytest.mark.parametrize("dist", [EXP, NORMAL])
@pytest.mark.parametrize("n", [8, 256])
def test_equal_areas_and_closure(O, dist, n):
    t = O.trad_arrays(dist, n)
    X, f, W, v = t["X"], t["f"], t["W"], t["v"]
    assert X[n - 1] == 0.0 and f[n - 1] == 1.0
    assert np.all(np.diff(X) < 0) and np.all(np.diff(f) > 0)
    # base: rectangle plus tail; layers i >= 1: width X_{i-1}, height f_i - f_{i-1}
    tail = math.exp(-X[0]) if dist == EXP else math.sqrt(math.pi / 2) * special.erfc(X[0] / math.sqrt(2))
    assert abs(X[0] * f[0] + tail - v) < 1e-15
    assert W[0] == v / f[0] or abs(W[0] - v / f[0]) < 1e-15 * W[0]
    for i in range(1, n):
        area = Fraction(W[i]) * (Fraction(f[i]) - Fraction(f[i - 1]))
        assert abs(float(area) - v) < 1e-13 * v, i
        assert W[i] == X[i - 1]
    dens = (lambda x: math.exp(-x)) if dist == EXP else (lambda x: math.exp(-0.5 * x * x))
    for i in range(n - 1):
        assert abs(f[i] - dens(X[i])) < 1e-15


@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_distribution(O, dist):
    x = O.trad_fill(dist, 3, 0, 4 * 10 ** 6, 1.0, 0.0, threads=8)
    assert stats.kstest(x, "expon" if dist == EXP else "norm").pvalue > P_MIN
    u = -np.expm1(-x) if dist == EXP else special.ndtr(x)
    h = np.bincount(np.minimum((u * 1000).astype(np.int64), 999), minlength=1000)
    assert stats.chisquare(h).pvalue > P_MIN
    for k in range(1, 5):
        if dist == EXP:
            mu, m2k = math.factorial(k), math.factorial(2 * k)
        else:
            mu = 0 if k % 2 else [1, 3][k // 2 - 1]
            m2k = [1, 3, 15, 105][k - 1]
        se = math.sqrt((m2k - mu * mu) / len(x))
        assert abs(np.mean(x ** k) - mu) < 4.5 * se, k


@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_small_stack_distribution_and_slow_share(O, dist):
    """With 8 layers most draws leave the quick path; the output must still
    follow the exact CDF, and the share of draws using slow words must be
    1 - mean(k_i) (each first draw quick-exits with probability k_i)."""
    x, w = O.trad_fill(dist, 5, 0, 2 * 10 ** 6, 1.0, 0.0, threads=8, layers=8, words=True)
    assert stats.kstest(x, "expon" if dist == EXP else "norm").pvalue > P_MIN
    k = O.trad_arrays(dist, 8)["k"].mean()
    share = (w > 0).mean()
    assert abs(share - (1 - k)) < 5 * math.sqrt(k * (1 - k) / len(x))
