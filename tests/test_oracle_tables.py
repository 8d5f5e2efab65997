"""Pins of the oracle's table construction (section 2 of the paper, its
layer equation, the overhang split after Table 1, Appendices B and D)
against values the paper prints, closed forms, invariants and an
independent high-precision recomputation."""
import math
import os

import mpmath as mp
import numpy as np
import pytest

import mp_tables

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_pins.txt")
IMAXES = [8, 16, 32, 64, 128, 256, 512, 1024]


def pins():
    d = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, rest = line.split(None, 1)
        d[name] = rest
    return d


def _P(dist, x):
    return mp.exp(-x) if dist == 0 else mp.exp(-x * x / 2)


def test_paper_layer_count(O):
    """L_max = 252 for the exponential at i_max = 256 (section 2)."""
    want = int(pins()["L_exp_256"].split()[0])
    assert O.table_arrays(0, 256)["L"] == want == 252


def test_1024_layer_counts(O):
    """Appendix D item 1's 1024 layers: four regions' worth of mass stays
    outside the layers for the exponential (L = 1020, 0.39 % slow draws)
    and three for the normal (L = 1021, 0.29 %); the independent mpmath
    construction confirms the counts."""
    assert O.table_arrays(0, 1024)["L"] == 1020
    assert O.table_arrays(1, 1024)["L"] == 1021


def test_paper_fast_exit_and_overhang_share(O):
    """98.4 % of draws exit on the fast path and the overhangs hold 4/256 =
    1.6 % of the mass (section 2, Table 1); under 2 % (Figure 1)."""
    t = O.table_arrays(0, 256)
    assert round(100 * t["L"] / 256, 1) == float(pins()["fast_exit_exp_256_percent"].split()[0])
    assert 256 - t["L"] == 4
    with mp.workdps(40):
        sumA = mp.fsum(mp.mpf(s) for s in t["hpA"])
        share = sumA / mp.mpf(t["hp_total"])
        assert abs(share - mp.mpf(4) / 256) < mp.mpf(10) ** -30
        assert share < mp.mpf(2) / 100
    tn = O.table_arrays(1, 256)
    assert (256 - tn["L"]) / 256 < 0.02


def test_paper_band_and_eliminated_tests(O):
    """The widest band between chord and curve is 9 % of the box height and
    the three-region split avoids 91 % of the rejection tests (paragraph
    after Table 1).  Without reflection the band covers eps - eps^2/2 of the
    unit box."""
    p = pins()
    eps = O.table_arrays(0, 256)["eps"]
    assert round(100 * eps) == int(p["band_height_percent"].split()[0])
    assert round(100 * (1 - (eps - eps * eps / 2))) == int(p["tests_eliminated_percent"].split()[0])


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", IMAXES)
def test_equal_area_and_stop_rule(O, dist, i_max):
    """Each layer has area exactly 1/i_max of the total: X_k (P(X_k) -
    P(X_{k-1})) = a (section 2), checked in 50-digit arithmetic from the
    113-bit values; and no further layer fits on top of the last one."""
    t = O.table_arrays(dist, i_max)
    L = t["L"]
    with mp.workdps(50):
        a = mp.mpf(t["hp_area"])
        tot = _P(0, 0) if dist == 0 else mp.sqrt(mp.pi / 2)
        assert abs(a - tot / i_max) < mp.mpf(10) ** -33
        fprev = mp.mpf(0)
        for k in range(L):
            X = mp.mpf(t["hpX"][k])
            fk = _P(dist, X)
            rel = abs(X * (fk - fprev) - a) / a
            assert rel < mp.mpf(10) ** -28, (k, rel)
            fprev = fk
        # stop rule: max_X X (P(X) - f_{L-1}) < a
        g = lambda x: x * (_P(dist, x) - fprev)
        xs = [mp.mpf(i) / 4000 * mp.mpf(t["hpX"][L - 1]) for i in range(1, 4001)]
        assert max(g(x) for x in xs) < a
    # the doubles are the rounded 113-bit values
    for k in range(L):
        assert t["X"][k] == float(mp.mpf(t["hpX"][k]))
        assert t["f"][k] == float(mp.mpf(t["hpf"][k]))


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", IMAXES)
def test_monotone_and_coverage(O, dist, i_max):
    """X strictly decreases and f strictly increases up the ziggurat; layers
    plus tail, overhangs and cap cover the total mass exactly, and the
    non-layer mass is (i_max - L)/i_max of it (section 2)."""
    t = O.table_arrays(dist, i_max)
    L = t["L"]
    X, f = t["X"][:L], t["f"][:L]
    assert np.all(np.diff(X) < 0) and np.all(np.diff(f) > 0)
    assert X[-1] > 0 and f[-1] < 1 and f[0] > 0
    with mp.workdps(50):
        a = mp.mpf(t["hp_area"])
        tot = mp.mpf(t["hp_total"])
        A = [mp.mpf(s) for s in t["hpA"]]
        assert all(v > 0 for v in A)
        assert abs(L * a + mp.fsum(A) - tot) / tot < mp.mpf(10) ** -30
        # region masses recomputed by direct quadrature from the 113-bit corners
        Xh = [mp.mpf(s) for s in t["hpX"][:L]] + [mp.mpf(0)]
        fh = [_P(dist, x) for x in Xh[:L]]
        tail = mp.quad(lambda x: _P(dist, x), [Xh[0], mp.inf])
        assert abs(tail - A[0]) / A[0] < mp.mpf(10) ** -25
        for j in sorted({1, L // 2, L - 1, L}):
            if j < 1:
                continue
            qv = mp.quad(lambda x: _P(dist, x) - fh[j - 1], [Xh[j], Xh[j - 1]])
            assert abs(qv - A[j]) / A[j] < mp.mpf(10) ** -25, j


@pytest.mark.parametrize("dist,i_max", [(0, 8), (1, 8), (0, 16), (1, 16), (0, 64), (1, 64), (0, 256), (1, 256),
                                        (0, 1024), (1, 1024)])
def test_independent_recomputation(O, dist, i_max):
    """A second construction (mpmath, solving for f by golden-section and
    bisection) rounds to the same doubles, bit for bit."""
    Xs, Fs, area, total = mp_tables.build(dist, i_max)
    t = O.table_arrays(dist, i_max)
    assert len(Xs) == t["L"]
    for k in range(len(Xs)):
        assert float(Xs[k]) == t["X"][k], k
        assert float(Fs[k]) == t["f"][k], k


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", [8, 16, 256, 512, 1024])
def test_derived_tables(O, dist, i_max):
    """Box widths and heights, the fast-path scale and its single-precision
    copy (the 32-bit word keeps s = max(b, 8) low bits for the index, so its
    magnitude has 32 - s bits for the exponential and 31 - s for the
    normal), the tail constants."""
    t = O.table_arrays(dist, i_max)
    L = t["L"]
    X, f = t["X"], t["f"]
    assert X[L] == 0.0 and f[L] == 1.0
    for j in range(1, L + 1):
        assert t["W"][j] == X[j - 1] - X[j]
        assert t["H"][j] == f[j] - f[j - 1]
        assert t["W"][j] > 0 and t["H"][j] > 0
    for i in range(L):
        assert t["XS"][i] == math.ldexp(X[i], -53)
        s32 = max(t["b"], 8)
        e = s32 - 32 if dist == 0 else s32 - 31
        assert t["XS32"][i] == np.float32(math.ldexp(float(np.float32(mp.mpf(t["hpX"][i]))), e))
    assert np.all(t["XS"][L:] == 0)
    assert t["X0"] == X[0]
    with mp.workdps(50):
        assert t["invX0"] == float(1 / mp.mpf(t["hpX"][0]))


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", IMAXES)
def test_alias_exact(O, dist, i_max):
    """The alias table reproduces the integer region weights exactly:
    sum_c T_c [c = j] + (cap - T_c) [alias_c = j] = q_j, the weights sum to
    2^64 and are the rounded region masses (section 2, O(1) draw of j)."""
    t = O.table_arrays(dist, i_max)
    L, b = t["L"], t["b"]
    cap = 1 << (64 - b)
    q = [int(v) for v in t["q"]]
    assert sum(q) == 1 << 64
    T = [int(v) for v in t["T"]]
    A = [int(v) for v in t["A"]]
    got = [0] * (L + 1)
    for c in range(i_max):
        assert 0 <= T[c] <= cap
        if c <= L:
            got[c] += T[c]
        else:
            assert T[c] == 0
        if T[c] < cap:
            assert A[c] <= L
            got[A[c]] += cap - T[c]
    assert got == q
    with mp.workdps(50):
        Am = [mp.mpf(s) for s in t["hpA"]]
        S = mp.fsum(Am)
        for j in range(L):
            assert abs(mp.mpf(q[j]) - Am[j] / S * mp.mpf(2) ** 64) <= mp.mpf("0.5000001")
    # the draw compares the high 64-b bits with the column threshold
    for c in range(i_max):
        if 0 < T[c] < cap:
            assert O.alias_draw(dist, i_max, c | ((T[c] - 1) << b)) == c
            assert O.alias_draw(dist, i_max, c | (T[c] << b)) == A[c]
        elif T[c] == cap:
            assert O.alias_draw(dist, i_max, c | ((cap - 1) << b)) == c
        else:
            assert O.alias_draw(dist, i_max, c) == A[c]


@pytest.mark.parametrize("i_max", IMAXES)
def test_eps_brute_force(O, i_max):
    """eps bounds the normalised gap between the chord and e^-x in every
    exponential box and is attained in the widest one: checked by dense
    evaluation of the gap, without the closed form."""
    t = O.table_arrays(0, i_max)
    L = t["L"]
    u = np.linspace(0.0, 1.0, 200001)
    best = 0.0
    best_j = -1
    for j in range(1, L + 1):
        X, W, H, fb = t["X"][j], t["W"][j], t["H"][j], t["f"][j - 1]
        curve = (np.exp(-(X + u * W)) - fb) / H
        gap = (1.0 - u) - curve
        m = gap.max()
        assert m <= t["eps"] + 1e-9, j
        if m > best:
            best, best_j = m, j
    assert abs(best - t["eps"]) < 1e-9
    widths = [t["W"][j] for j in range(1, L + 1)]
    assert best_j == 1 + int(np.argmax(widths))
    with mp.workdps(40):
        eps = mp.mpf(t["hp_eps"])
        assert t["K_eps"] == int(mp.floor((1 - eps) * mp.mpf(2) ** 53))
