"""Pins of the oracle's sampler (Table 1's modified column, the tail
samplers and the overhang split of the paper) against brute force on
lattices, exact conditional CDFs, closed-form moments and the paper's
Appendix B moments."""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

P_MIN = 1e-4  # seeded inputs: a fixed sample passes or fails deterministically


def _box(t, j):
    return t["X"][j], t["W"][j], t["H"][j], t["f"][j - 1]


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _under_exact(dist, x, y):
    with mp.workdps(40):
        xv, yv = mp.mpf(x), mp.mpf(y)
        p = mp.exp(-xv) if dist == 0 else mp.exp(-xv * xv / 2)
        return yv < p, abs(p - yv)


def _brute(dist, t, j, g):
    """For every lattice point (a, c) of the g x g grid in box j: where the
    sampler must land (mirror image across the chord for exponential
    points above it) and whether that point lies under P."""
    Xl, W, H, fb = _box(t, j)
    a = np.arange(g)[:, None] * np.ones((1, g), dtype=np.int64)
    c = np.ones((g, 1), dtype=np.int64) * np.arange(g)[None, :]
    if dist == 0:
        up = (a + c) > g
        ra = np.where(up, g - c, a)
        rc = np.where(up, g - a, c)
    else:
        ra, rc = a, c
    xs = np.array([_fma(k / g, W, Xl) for k in range(g + 1)])
    ys = np.array([_fma(k / g, H, fb) for k in range(g + 1)])
    x = xs[ra]
    y = ys[rc]
    p = np.exp(-x) if dist == 0 else np.exp(-0.5 * x * x)
    under = y < p
    close = np.abs(p - y) < 1e-9
    near = np.zeros_like(under)
    for ia, ic in zip(*np.nonzero(close)):
        u, gap = _under_exact(dist, x[ia, ic], y[ia, ic])
        under[ia, ic] = u
        near[ia, ic] = gap < mp.mpf(2) ** -40
    return under, x, near


BOXES = [(0, 8, None), (1, 8, None), (0, 256, [1, 2, 126, 251, 252]), (1, 256, [1, "straddle", 126, 252, 253])]


@pytest.mark.parametrize("dist,i_max,js", BOXES)
def test_box_lattice_brute_force(O, dist, i_max, js):
    """Every attempt on a 512 x 512 lattice: the oracle accepts exactly the
    points that lie under P after the reflection of the exponential
    overhang (Appendix C item 5), its eps shortcut never accepts a point
    above P, and the returned x is the abscissa of that point."""
    t = O.table_arrays(dist, i_max)
    L = t["L"]
    if js is None:
        js = list(range(1, L + 1))
    g = 512
    shift = 53 - 9
    for j in js:
        if j == "straddle":
            j = next(k for k in range(1, L) if t["X"][k] < 1.0 < t["X"][k - 1])
        acc, xo = O.box_grid(dist, i_max, j, g, shift)
        under, xb, near = _brute(dist, t, j, g)
        far = ~near
        assert np.array_equal(acc[far], under[far]), (j, int((acc[far] != under[far]).sum()))
        assert np.array_equal(xo[acc], xb[acc])
        assert acc.mean() > 0.3


def test_box_eps_shortcut_region(O):
    """Points strictly inside the fast-accept triangle are accepted without
    a P evaluation, those on the chord band are tested: the shortcut fires
    exactly when k1 + k2 <= K_eps."""
    t = O.table_arrays(0, 256)
    K = t["K_eps"]
    one = 1 << 53
    ok, x = O.box_attempt(0, 256, 1, K // 2, K - K // 2)
    assert ok
    # a point just above the chord maps onto its mirror just below it
    ok1, x1 = O.box_attempt(0, 256, 1, one // 2 + 5, one // 2)
    ok2, x2 = O.box_attempt(0, 256, 1, one // 2, one // 2 - 5)
    assert ok1 == ok2 and (not ok1 or x1 == x2)


def _exp_box_cdf(t, j, x):
    Xl, W, H, fb = _box(t, j)
    x = np.asarray(x)
    el = math.exp(-Xl)
    num = -el * np.expm1(-(x - Xl)) - fb * (x - Xl)
    den = -el * math.expm1(-W) - fb * W
    return num / den


def _norm_int(a, b):
    """integral of e^-t^2/2 from a to b (vectorised over b)"""
    s = math.sqrt(math.pi / 2)
    return s * (special.erfc(a / math.sqrt(2)) - special.erfc(np.asarray(b) / math.sqrt(2)))


def _norm_box_cdf(t, j, x):
    Xl, W, H, fb = _box(t, j)
    x = np.asarray(x)
    return (_norm_int(Xl, x) - fb * (x - Xl)) / (_norm_int(Xl, Xl + W) - fb * W)


@pytest.mark.parametrize("dist,i_max,js", BOXES)
def test_box_conditional_distribution(O, dist, i_max, js):
    """Conditional on region j, x has density proportional to P(x) -
    f_{j-1} on [X_j, X_{j-1}] (section 2, overhang areas A_i)."""
    t = O.table_arrays(dist, i_max)
    L = t["L"]
    if js is None:
        js = list(range(1, L + 1))
    for j in js:
        if j == "straddle":
            j = next(k for k in range(1, L) if t["X"][k] < 1.0 < t["X"][k - 1])
        x = O.sample_region(dist, j, seed=1000 + j, index0=0, n=100000, i_max=i_max)
        Xl, W = t["X"][j], t["W"][j]
        assert x.min() >= Xl and x.max() <= Xl + W
        cdf = (lambda v: _exp_box_cdf(t, j, v)) if dist == 0 else (lambda v: _norm_box_cdf(t, j, v))
        p = stats.kstest(x, cdf).pvalue
        assert p > P_MIN, (j, p)


def _norm_tail_sf(x):
    return special.erfc(np.asarray(x) / math.sqrt(2)) / 2


@pytest.mark.parametrize("i_max", [8, 256])
def test_exp_tail(O, i_max):
    """The exponential tail is X_0 plus an Exp(1) variate (memorylessness,
    the paragraph after Table 1): x - X_0 ~ Exp(1)."""
    t = O.table_arrays(0, i_max)
    x = O.sample_region(0, 0, seed=77, index0=0, n=400000, i_max=i_max)
    d = x - t["X0"]
    assert d.min() >= 0
    assert stats.kstest(d, "expon").pvalue > P_MIN
    assert abs(d.mean() - 1) < 4 / math.sqrt(len(d))


@pytest.mark.parametrize("i_max", [8, 256])
def test_normal_tail(O, i_max):
    """The normal tail (Marsaglia's method on exponential draws) has CDF
    1 - Q(x)/Q(X_0) on x >= X_0, Q the standard normal upper tail."""
    t = O.table_arrays(1, i_max)
    X0 = t["X0"]
    x = O.sample_region(1, 0, seed=78, index0=0, n=400000, i_max=i_max)
    assert x.min() >= X0
    qx0 = _norm_tail_sf(X0)
    cdf = lambda v: 1 - _norm_tail_sf(v) / qx0
    assert stats.kstest(x, cdf).pvalue > P_MIN


@pytest.mark.parametrize("dist", [0, 1])
def test_tail_quantiles_by_inversion(O, dist):
    """Empirical tail quantiles at tiny tables (i_max = 8) against the exact
    tail CDF inverted by bisection."""
    t = O.table_arrays(dist, 8)
    X0 = t["X0"]
    n = 200000
    x = np.sort(O.sample_region(dist, 0, seed=79, index0=5, n=n, i_max=8))
    with mp.workdps(30):
        if dist == 0:
            F = lambda v: 1 - mp.exp(-(v - X0))
            dens = lambda v: mp.exp(-(v - X0))
        else:
            q0 = mp.erfc(X0 / mp.sqrt(2))
            F = lambda v: 1 - mp.erfc(v / mp.sqrt(2)) / q0
            dens = lambda v: mp.sqrt(2 / mp.pi) * mp.exp(-v * v / 2) / q0
        for p in [0.01, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99]:
            lo, hi = mp.mpf(X0), mp.mpf(X0) + 60
            for _ in range(120):
                mid = (lo + hi) / 2
                if F(mid) < p:
                    lo = mid
                else:
                    hi = mid
            qv = float(lo)
            emp = x[int(p * n)]
            se = math.sqrt(p * (1 - p) / n) / float(dens(lo))
            assert abs(emp - qv) < 5 * se, (p, emp, qv, se)


def _cdf(dist, x):
    if dist == 0:
        return -np.expm1(-x)
    return special.ndtr(x)


def _moments_ok(dist, x, scale=1.0, shift=0.0):
    z = (x.astype(np.float64) - shift) / scale
    n = len(z)
    for k in range(1, 6):
        m = np.mean(z ** k)
        if dist == 0:
            mu, m2k = math.factorial(k), math.factorial(2 * k)
        else:
            dfact = lambda r: 1 if r <= 0 else r * dfact(r - 2)
            mu = 0 if k % 2 else dfact(k - 1)
            m2k = dfact(2 * k - 1)
        se = math.sqrt((m2k - mu * mu) / n)
        assert abs(m - mu) < 4.5 * se, (k, m, mu, se)


def _chi2_equiprobable(u, bins=10000):
    h = np.bincount(np.minimum((u * bins).astype(np.int64), bins - 1), minlength=bins)
    return stats.chisquare(h).pvalue


@pytest.mark.slow
@pytest.mark.parametrize("dist,seed", [(0, 1), (1, 7)])
def test_whole_distribution_1e8(O, dist, seed):
    """10^8 FP64 draws: KS and chi-square (10^4 equiprobable bins through the
    exact CDF) against Exp(1) / N(0,1), raw moments 1..5 against m! and
    0,1,0,3,0 within 4.5 standard errors (Appendix B; errors scale as
    1/sqrt(N))."""
    n = 10 ** 8
    x = O.fill(dist, 0, seed, 0, n, 1.0, 0.0, threads=8)
    if dist == 0:
        assert x.min() >= 0
    u = _cdf(dist, x)
    assert _chi2_equiprobable(u) > P_MIN
    u.sort()
    i = np.arange(1, n + 1, dtype=np.float64)
    D = max(np.max(i / n - u), np.max(u - (i - 1) / n))
    del i
    p = stats.kstwo.sf(D, n)
    assert p > P_MIN, (D, p)
    _moments_ok(dist, x)


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", [8, 16])
def test_small_tables_whole_distribution(O, dist, i_max):
    """With 8 or 16 layers the slow paths carry 12-40 % of the draws; the
    output must still follow the exact CDF."""
    x = O.fill(dist, 0, 11, 0, 2 * 10 ** 6, 1.0, 0.0, threads=8, i_max=i_max)
    assert stats.kstest(x, "expon" if dist == 0 else "norm").pvalue > P_MIN
    assert _chi2_equiprobable(_cdf(dist, x), 1000) > P_MIN
    _moments_ok(dist, x)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("dist", [0, 1])
def test_1024_layers_whole_distribution(O, dist, dtype):
    """Appendix D item 1's 1024 layers, in both output types: exact CDF
    and moments."""
    x = O.fill(dist, dtype, 13, 5, 4 * 10 ** 6, 1.0, 0.0, threads=8, i_max=1024).astype(np.float64)
    assert stats.kstest(x, "expon" if dist == 0 else "norm").pvalue > P_MIN
    assert _chi2_equiprobable(_cdf(dist, x), 1000) > P_MIN
    _moments_ok(dist, x)


@pytest.mark.parametrize("dist", [0, 1])
def test_fp32_bits_at_1024_layers(O, dist):
    """With 10 index bits the single-precision magnitude starts at bit 10
    (exponential, 22 bits) or 11 (normal, sign at bit 10, 21 bits): on the
    fast path k = |x| / XS32_i is an integer below 2^(32-10) or 2^(31-10),
    uniform, and its low bits are independent of the index bits 8..9 (a
    magnitude that reused index bits would tie them together)."""
    n = 10 ** 6
    t = O.table_arrays(dist, 1024)
    out, layer, region, words, tests = O.fill_trace(dist, 1, 17, 0, n, 1.0, 0.0, i_max=1024)
    fast = region < 0
    xs32 = t["XS32"].astype(np.float64)
    kf = np.abs(out[fast].astype(np.float64)) / xs32[layer[fast]]
    k = np.rint(kf).astype(np.int64)
    assert np.all(np.abs(kf - k) < 0.25)
    bits = 22 if dist == 0 else 21
    assert k.min() >= 0 and k.max() < 2 ** bits and k.max() >= 2 ** bits - 2 ** (bits - 6)
    assert stats.chisquare(np.bincount(k >> (bits - 8), minlength=256)).pvalue > P_MIN
    table = np.zeros((4, 4))
    np.add.at(table, ((layer[fast] >> 8) & 3, k & 3), 1)
    assert stats.chi2_contingency(table)[1] > P_MIN
    if dist == 1:
        assert abs((out < 0).mean() - 0.5) < 4.5 * 0.5 / math.sqrt(n)
        sign = np.zeros((4, 2))
        np.add.at(sign, ((layer[fast] >> 8) & 3, (out[fast] < 0).astype(np.int64)), 1)
        assert stats.chi2_contingency(sign)[1] > P_MIN


@pytest.mark.parametrize("dist", [0, 1])
def test_fp32_distribution(O, dist):
    x = O.fill(dist, 1, 21, 3, 4 * 10 ** 6, 1.0, 0.0, threads=8)
    assert x.dtype == np.float32
    assert stats.kstest(x.astype(np.float64), "expon" if dist == 0 else "norm").pvalue > P_MIN
    _moments_ok(dist, x)


@pytest.mark.parametrize("dtype", [0, 1])
def test_location_scale(O, dtype):
    """Exp(lambda = 2.5): mean 1/lambda, variance 1/lambda^2; N(-1, 3^2)."""
    n = 2 * 10 ** 6
    lam = 2.5
    x = O.fill(0, dtype, 11, 0, n, 1.0 / lam, 0.0, threads=8).astype(np.float64)
    assert abs(x.mean() - 1 / lam) < 4.5 * (1 / lam) / math.sqrt(n)
    assert stats.kstest(x, "expon", args=(0, 1 / lam)).pvalue > P_MIN
    y = O.fill(1, dtype, 12, 0, n, 3.0, -1.0, threads=8).astype(np.float64)
    assert abs(y.mean() + 1) < 4.5 * 3 / math.sqrt(n)
    assert stats.kstest(y, "norm", args=(-1, 3)).pvalue > P_MIN


@pytest.mark.parametrize("dist", [0, 1])
def test_fast_path_layers_and_regions(O, dist):
    """Layer index uniform over i_max; fast exits at rate L/i_max; on the
    fast path x/X_i uniform on [0,1) (Table 1 step 2); slow draws select
    region j with probability q_j / 2^64."""
    n = 10 ** 6
    t = O.table_arrays(dist, 256)
    L = t["L"]
    out, layer, region, words, tests = O.fill_trace(dist, 0, 31, 0, n, 1.0, 0.0)
    assert stats.chisquare(np.bincount(layer, minlength=256)).pvalue > P_MIN
    fast = region < 0
    assert np.array_equal(fast, layer < L)
    pf = L / 256
    assert abs(fast.mean() - pf) < 4.5 * math.sqrt(pf * (1 - pf) / n)
    u = np.abs(out[fast]) / t["X"][layer[fast]]
    assert u.min() >= 0 and u.max() < 1
    assert stats.kstest(u, "uniform").pvalue > P_MIN
    j = region[~fast]
    q = t["q"].astype(np.float64) / 2.0 ** 64
    h = np.bincount(j, minlength=L + 1)
    exp_counts = q * len(j)
    keep = exp_counts >= 5
    f_obs, f_exp = h[keep], exp_counts[keep]
    if exp_counts[~keep].sum() > 0:
        f_obs = np.append(f_obs, h[~keep].sum())
        f_exp = np.append(f_exp, exp_counts[~keep].sum())
    f_exp *= f_obs.sum() / f_exp.sum()
    assert stats.chisquare(f_obs, f_exp).pvalue > P_MIN
    if dist == 1:
        assert abs((out < 0).mean() - 0.5) < 4.5 * 0.5 / math.sqrt(n)


def test_exp_shortcut_rate(O):
    """Exponential overhang attempts are reflected into the lower triangle,
    where only the band 1 - eps < u + v <= 1 needs exp(): with one global
    eps every box calls it on a fraction 2 eps - eps^2 of its attempts (the
    paragraph after Table 1, Appendix C item 5, Appendix D item 2)."""
    t = O.table_arrays(0, 256)
    eps = t["eps"]
    out, layer, region, words, tests = O.fill_trace(0, 0, 32, 0, 4 * 10 ** 6, 1.0)
    box = region > 0
    attempts = int(((words[box] - 1) // 2).sum())
    p = 2 * eps - eps * eps
    rate = tests[box].sum() / attempts
    assert abs(rate - p) < 4.5 * math.sqrt(p * (1 - p) / attempts), (rate, p, attempts)
