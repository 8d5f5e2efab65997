"""Pins of the oracle's raw-moment sums (the fused generate-and-reduce
form): the fixed summation order stays within the proven error bound of
the correctly rounded sum (math.fsum) of the same powers, the result does
not depend on the thread count, empty and one-output ranges, FP32 outputs
widened before the powers, and the sample moments against the closed forms
E[X^p] = p!/lambda^p (exponential) and the normal raw moments (Appendix B
tabulates X1..X5 of 10^12 draws against 1, 2, 6, 24, 120 and 0, 1, 0, 3, 0)."""
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


def order_depth(n, per):
    """Longest chain of additions in the fixed order: a lane adds at most
    8 * per outputs, then 8 halving levels over lanes, 8 over tiles, then
    the groups one after the other."""
    tiles = -(-n // (2048 * per)) + 1
    groups = -(-tiles // 256)
    return 8 * per + 8 + 8 + groups + 1


@pytest.mark.parametrize("dist,dtype,first,n,p0,p1", [
    (EXP, F64, 0, 1_000_003, 1.0, 0.0), (NORMAL, F64, 7, 600_001, -1.0, 3.0),
    (EXP, F32, 3, 900_000, 2.5, 0.0), (NORMAL, F32, 2 ** 40 + 1, 555_555, 0.5, 0.25),
    (EXP, F64, 1, 4096 * 300 + 17, 0.3, 0.0)])
def test_fixed_order_within_bound_of_exact_sum(O, dist, dtype, first, n, p0, p1):
    scale, shift = (1.0 / p0, 0.0) if dist == EXP else (p1, p0)
    got = O.moments(dist, dtype, 42, first, n, scale, shift, threads=8)
    x = O.fill(dist, dtype, 42, first, n, scale, shift, threads=8)
    per = 2 if dtype == F64 else 4
    h = order_depth(n, per)
    u = 2.0 ** -53
    gamma = h * u / (1 - h * u)
    for p, q in enumerate(powers(x)):
        exact = math.fsum(q)
        bound = gamma * math.fsum(np.abs(q)) + 1e-300
        assert abs(got[p] - exact) <= bound, (p, got[p], exact, bound)


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
