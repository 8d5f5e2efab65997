"""Pins of the oracle's raw-moment sums (Appendix B's statistic, section
3's generate-and-aggregate form).

The oracle adds every term exactly and rounds once, so its sums must equal
Python's math.fsum (Shewchuk's correctly rounded summation, an independent
algorithm) bit for bit: first on hand-made and random arrays that stress
rounding (ties, cancellation, subnormals, wide exponent ranges), then on
the powers of the oracle's own fill outputs.  The sample moments are
checked against the closed forms E[X^p] = p!/lambda^p (exponential) and
the normal raw moments (Appendix B tabulates X1..X5 of 10^12 draws against
1, 2, 6, 24, 120 and 0, 1, 0, 3, 0)."""
import math

import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL


def powers(x):
    x = x.astype(np.float64)
    q2 = x * x
    q3 = q2 * x
    q4 = q2 * q2
    q5 = q4 * x
    return [x, q2, q3, q4, q5]


def bits(v):
    return np.float64(v).view(np.uint64)


@pytest.mark.parametrize("xs,want", [
    ([], 0.0),
    ([2.5], 2.5),
    ([1.0, 2.0 ** -53], 1.0),                          # tie, to even (down)
    ([1.0 + 2.0 ** -52, 2.0 ** -53], 1.0 + 2.0 ** -51),  # tie, to even (up)
    ([1.0, 2.0 ** -53, 2.0 ** -105], 1.0 + 2.0 ** -52),  # just above the tie
    ([1.0, -(2.0 ** -53)], 1.0 - 2.0 ** -53),          # exact below 1
    ([1.0, -(2.0 ** -54)], 1.0),                        # tie below 1, to even
    ([1.0, -(2.0 ** -54), -(2.0 ** -200)], 1.0 - 2.0 ** -53),
    ([1e300, 1.0, -1e300], 1.0),                        # cancellation
    ([5e-324, 5e-324, -5e-324], 5e-324),               # subnormals
    ([2.0 ** -1022, -(2.0 ** -1074)], 2.0 ** -1022 - 2.0 ** -1074),
    ([1.0, -1.0], 0.0),
])
def test_exact_sum_hand_cases(O, xs, want):
    got = O.exact_sum(np.array(xs, dtype=np.float64))
    assert bits(got) == bits(want), (xs, got, want)


def test_exact_sum_zero_is_positive(O):
    assert bits(O.exact_sum(np.array([-0.0]))) == bits(0.0)
    assert bits(O.exact_sum(np.array([3.0, -3.0]))) == bits(0.0)


@pytest.mark.parametrize("seed", range(8))
def test_exact_sum_equals_fsum(O, seed):
    rng = np.random.default_rng(seed)
    for _ in range(50):
        n = int(rng.integers(1, 3000))
        span = int(rng.choice([4, 60, 400, 1500]))
        e = rng.integers(-span, span, n)
        x = rng.standard_normal(n) * np.exp2(np.clip(e, -1070, 1000).astype(np.float64))
        if rng.random() < 0.3:  # near-cancelling tails
            x = np.concatenate([x, -x[: n // 2] * (1 + 2.0 ** -52)])
        rng.shuffle(x)
        got = O.exact_sum(x)
        want = math.fsum(x)
        assert bits(got) == bits(want) or (got == 0.0 and want == 0.0), (got, want)


@pytest.mark.parametrize("dist,dtype,first,n,p0,p1", [
    (EXP, F64, 0, 1_000_003, 1.0, 0.0), (NORMAL, F64, 7, 600_001, -1.0, 3.0),
    (EXP, F32, 3, 900_000, 2.5, 0.0), (NORMAL, F32, 2 ** 40 + 1, 555_555, 0.5, 0.25),
    (EXP, F64, 1, 4096 * 300 + 17, 0.3, 0.0)])
def test_moments_equal_fsum_of_fill_powers(O, dist, dtype, first, n, p0, p1):
    scale, shift = (1.0 / p0, 0.0) if dist == EXP else (p1, p0)
    got, gabs = O.moments(dist, dtype, 42, first, n, scale, shift, threads=8, with_abs=True)
    x = O.fill(dist, dtype, 42, first, n, scale, shift, threads=8)
    for p, q in enumerate(powers(x)):
        assert bits(got[p]) == bits(math.fsum(q)), (p, got[p], math.fsum(q))
        assert bits(gabs[p]) == bits(math.fsum(np.abs(q))), p


def test_thread_count_does_not_matter(O):
    a = O.moments(NORMAL, F64, 9, 11, 2_000_001, 2.0, 1.0, threads=1)
    b = O.moments(NORMAL, F64, 9, 11, 2_000_001, 2.0, 1.0, threads=7)
    assert a.tobytes() == b.tobytes()


def test_empty_and_single(O):
    assert O.moments(EXP, F64, 1, 5, 0, 1.0).tolist() == [0.0] * 5
    x = O.fill(NORMAL, F32, 1, 5, 1, 1.0, 0.0)
    d = float(np.float64(x[0]))
    q2 = d * d
    want = [d, q2, q2 * d, q2 * q2, (q2 * q2) * d]
    assert O.moments(NORMAL, F32, 1, 5, 1, 1.0, 0.0).tolist() == want


@pytest.mark.parametrize("dist,lam_or_mu,sigma", [(EXP, 1.0, 0.0), (EXP, 2.5, 0.0), (NORMAL, 0.0, 1.0),
                                                  (NORMAL, -1.0, 3.0)])
def test_sample_moments_match_closed_forms(O, dist, lam_or_mu, sigma):
    n = 20_000_000
    if dist == EXP:
        lam = lam_or_mu
        m = [math.factorial(p) / lam ** p for p in range(1, 11)]
        got = O.moments(EXP, F64, 77, 0, n, 1.0 / lam, 0.0, threads=8) / n
    else:
        mu, s = lam_or_mu, sigma

        # raw moments of N(mu, s^2): sum over even k of C(p,k) mu^(p-k) s^k (k-1)!!
        def raw(p):
            return sum(math.comb(p, k) * mu ** (p - k) * s ** k * math.prod(range(k - 1, 0, -2))
                       for k in range(0, p + 1, 2))
        m = [raw(p) for p in range(1, 11)]
        got = O.moments(NORMAL, F64, 77, 0, n, s, mu, threads=8) / n
    for p in range(1, 6):
        sd = math.sqrt(max(m[2 * p - 1] - m[p - 1] ** 2, 0.0) / n)
        assert abs(got[p - 1] - m[p - 1]) <= 6 * sd + 1e-12, (p, got[p - 1], m[p - 1], sd)
