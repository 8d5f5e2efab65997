"""An independent high-precision construction of the ziggurat layers, used
only by the tests to pin the oracle's tables.

It differs from the oracle on purpose: it works in mpmath (decimal
precision, not binary128), and it solves each layer for its height f
instead of its length X (X(f) = -ln f for e^-x, sqrt(-2 ln f) for
e^-x^2/2), bracketing the maximum by golden-section search and the root
by bisection in f.
"""
import mpmath as mp

_GOLD = None


def build(dist, i_max, dps=45):
    global _GOLD
    with mp.workdps(dps):
        if dist == 0:
            x_of_f = lambda f: -mp.log(f)
            total = mp.mpf(1)
        else:
            x_of_f = lambda f: mp.sqrt(-2 * mp.log(f))
            total = mp.sqrt(mp.pi / 2)
        area = total / i_max
        r = (3 - mp.sqrt(5)) / 2
        Xs, Fs = [], []
        fprev = mp.mpf(0)
        while True:
            h = lambda f: x_of_f(f) * (f - fprev)
            lo, hi = fprev, mp.mpf(1)
            a, b = lo + r * (hi - lo), hi - r * (hi - lo)
            ha, hb = h(a), h(b)
            for _ in range(130):
                if ha < hb:
                    lo, a, ha = a, b, hb
                    b = hi - r * (hi - lo)
                    hb = h(b)
                else:
                    hi, b, hb = b, a, ha
                    a = lo + r * (hi - lo)
                    ha = h(a)
            fm = a if ha >= hb else b
            if h(fm) < area:
                break
            lo = fprev if fprev > 0 else mp.mpf(10) ** (-dps)
            hi = fm
            for _ in range(int(dps * 3.33) + 20):
                mid = (lo + hi) / 2
                if h(mid) < area:
                    lo = mid
                else:
                    hi = mid
            fk = (lo + hi) / 2
            Xs.append(x_of_f(fk))
            Fs.append(fk)
            fprev = fk
        return Xs, Fs, area, total
