"""Pins of the oracle's accelerated normal-overhang variant: convex boxes
(right of the inflection point) reflect points above the chord and accept
below an eps band, concave boxes (left of it, and the cap) accept below the
chord and reject above a delta band, the straddling box keeps plain
rejection.  Checked against: the band widths recomputed independently (a
golden-section search of the chord-curve gap in 50-digit arithmetic), a
lattice brute force of every attempt against the exact density, the exact
conditional distribution in each box, the whole N(0, 1) distribution, and
fewer attempts and density evaluations than plain rejection."""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

from helpers import F64, NORMAL

P_MIN = 1e-4


def _cls(t, j):
    if t["X"][j] >= 1.0:
        return "convex"
    if t["X"][j - 1] <= 1.0:
        return "concave"
    return "straddle"


def _gap_max(t, j, convex):
    """max over u of the normalised chord-curve gap, by golden section on
    the gap itself (the oracle solves for the slope instead)."""
    with mp.workdps(50):
        left = mp.mpf(t["hpX"][j]) if j < t["L"] else mp.mpf(0)
        right = mp.mpf(t["hpX"][j - 1])
        base = mp.mpf(t["hpf"][j - 1])
        top = mp.mpf(t["hpf"][j]) if j < t["L"] else mp.mpf(1)
        w, h = right - left, top - base

        def gap(u):
            c = (mp.exp(-(left + u * w) ** 2 / 2) - base) / h
            return (1 - u) - c if convex else c - (1 - u)

        a, b = mp.mpf(0), mp.mpf(1)
        r = (mp.sqrt(5) - 1) / 2
        for _ in range(160):
            m1, m2 = b - r * (b - a), a + r * (b - a)
            if gap(m1) < gap(m2):
                a = m1
            else:
                b = m2
        return gap((a + b) / 2)


@pytest.mark.parametrize("i_max", [8, 256])
def test_band_widths_independently(O, i_max):
    t = O.table_arrays(NORMAL, i_max)
    L = t["L"]
    classes = [_cls(t, j) for j in range(1, L + 1)]
    if i_max == 256:
        assert (classes.count("convex"), classes.count("concave"), classes.count("straddle")) == (203, 49, 1)
    eps = max(_gap_max(t, j, True) for j in range(1, L + 1) if classes[j - 1] == "convex")
    dlt = max(_gap_max(t, j, False) for j in range(1, L + 1) if classes[j - 1] == "concave")
    with mp.workdps(50):
        assert abs(mp.mpf(t["hp_eps_cvx"]) - eps) < mp.mpf(10) ** -28
        assert abs(mp.mpf(t["hp_del_ccv"]) - dlt) < mp.mpf(10) ** -28
        widen = 1 + mp.mpf(2) ** -20
        assert t["K_cvx"] == int(mp.floor((1 - eps * widen) * mp.mpf(2) ** 53))
        assert t["K_ccv"] == int(mp.ceil((1 + dlt * widen) * mp.mpf(2) ** 53))


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _brute(t, j, g):
    Xl, W, H, fb = t["X"][j], t["W"][j], t["H"][j], t["f"][j - 1]
    a = np.arange(g)[:, None] * np.ones((1, g), dtype=np.int64)
    c = np.ones((g, 1), dtype=np.int64) * np.arange(g)[None, :]
    if _cls(t, j) == "convex":
        up = (a + c) > g
        ra, rc = np.where(up, g - c, a), np.where(up, g - a, c)
    else:
        ra, rc = a, c
    xs = np.array([_fma(k / g, W, Xl) for k in range(g + 1)])
    ys = np.array([_fma(k / g, H, fb) for k in range(g + 1)])
    x, y = xs[ra], ys[rc]
    p = np.exp(-0.5 * x * x)
    under = y < p
    near = np.abs(p - y) < 1e-9
    for ia, ic in zip(*np.nonzero(near)):
        with mp.workdps(40):
            pv = mp.exp(-mp.mpf(x[ia, ic]) ** 2 / 2)
            under[ia, ic] = mp.mpf(y[ia, ic]) < pv
            near[ia, ic] = abs(pv - mp.mpf(y[ia, ic])) < mp.mpf(2) ** -40
    return under, x, near


@pytest.mark.parametrize("i_max,js", [(8, None), (256, [1, 100, 203, "straddle", 205, 230, 252, 253])])
def test_box_lattice_brute_force(O, i_max, js):
    """Every attempt on a 512 x 512 lattice: the variant accepts exactly the
    points under P (after the reflection in convex boxes), so its band
    shortcuts never change a decision, and returns that point's abscissa."""
    t = O.table_arrays(NORMAL, i_max)
    L = t["L"]
    if js is None:
        js = list(range(1, L + 1))
    g = 512
    for j in js:
        if j == "straddle":
            j = next(k for k in range(1, L) if _cls(t, k) == "straddle")
        acc, xo = O.box_grid(NORMAL, i_max, j, g, 53 - 9, accel=True)
        under, xb, near = _brute(t, j, g)
        far = ~near
        assert np.array_equal(acc[far], under[far]), (j, int((acc[far] != under[far]).sum()))
        assert np.array_equal(xo[acc], xb[acc])


def _norm_int(a, b):
    s = math.sqrt(math.pi / 2)
    return s * (special.erfc(a / math.sqrt(2)) - special.erfc(np.asarray(b) / math.sqrt(2)))


@pytest.mark.parametrize("i_max,js", [(8, None), (256, [1, 150, "straddle", 240, 253])])
def test_box_conditional_distribution(O, i_max, js):
    t = O.table_arrays(NORMAL, i_max)
    L = t["L"]
    if js is None:
        js = list(range(1, L + 1))
    for j in js:
        if j == "straddle":
            j = next(k for k in range(1, L) if _cls(t, k) == "straddle")
        x = O.sample_region(NORMAL, j, seed=2000 + j, index0=0, n=100000, i_max=i_max, accel=True)
        Xl, W, fb = t["X"][j], t["W"][j], t["f"][j - 1]
        assert x.min() >= Xl and x.max() <= Xl + W
        cdf = lambda v: (_norm_int(Xl, v) - fb * (np.asarray(v) - Xl)) / (_norm_int(Xl, Xl + W) - fb * W)
        assert stats.kstest(x, cdf).pvalue > P_MIN, j


@pytest.mark.parametrize("i_max", [8, 256])
def test_whole_distribution(O, i_max):
    n = 4 * 10 ** 6 if i_max == 256 else 2 * 10 ** 6
    x = O.fill(NORMAL, F64, 5, 0, n, 1.0, 0.0, threads=8, i_max=i_max, accel=True)
    assert stats.kstest(x, "norm").pvalue > P_MIN
    h = np.bincount(np.minimum((special.ndtr(x) * 1000).astype(np.int64), 999), minlength=1000)
    assert stats.chisquare(h).pvalue > P_MIN
    for k, mu in [(1, 0.0), (2, 1.0), (3, 0.0), (4, 3.0)]:
        m2k = [1, 3, 15, 105][k - 1]
        se = math.sqrt((m2k - mu * mu) / n)
        assert abs(np.mean(x ** k) - mu) < 4.5 * se, k


def test_fast_path_unchanged_and_fewer_attempts(O):
    """The variant changes only the overhang boxes: fast-path outputs and
    tails are the same as plain rejection's, and boxes take fewer slow
    words and far fewer density evaluations."""
    n = 3 * 10 ** 6
    a, la, ra, wa, ta = O.fill_trace(NORMAL, F64, 9, 0, n, 1.0, 0.0)
    b, lb, rb, wb, tb = O.fill_trace(NORMAL, F64, 9, 0, n, 1.0, 0.0, accel=True)
    assert np.array_equal(la, lb) and np.array_equal(ra, rb)
    fast = ra < 0
    assert np.array_equal(a[fast], b[fast])
    tail = ra == 0
    assert np.array_equal(a[tail], b[tail])
    box = ra > 0
    words_plain, words_acc = wa[box].mean(), wb[box].mean()
    tests_plain, tests_acc = ta[box].mean(), tb[box].mean()
    assert words_acc < words_plain and tests_acc < 0.5 * tests_plain, (words_plain, words_acc, tests_plain, tests_acc)
