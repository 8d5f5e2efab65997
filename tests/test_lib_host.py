"""Host-side checks of the library (no GPU needed): it loads, exports every
symbol include/zig.h declares, builds tables bit-identical to the oracle's
independent construction, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

from helpers import EXP, NORMAL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zig.h")


@pytest.fixture(scope="module")
def zig():
    from paper_1403_6870_amd import zig as z
    return z


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(zig_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(zig):
    names = declared_functions()
    assert "zig_fill_exp" in names and "zig_fill_normal" in names and "zig_build_tables" in names
    lib = ctypes.CDLL(zig.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert zig.zig_version().startswith("zigrand")


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_tables_match_oracle(zig, O, dist, i_max):
    """The library's binary128 construction (bracketed Newton) and the
    oracle's (bisection) give the same doubles and integers."""
    a = zig.zig_get_tables(dist, i_max)
    b = O.table_arrays(dist, i_max)
    assert a["L"] == b["L"]
    for k in ["X", "f", "XS", "XS32", "W", "H", "q", "T", "A"]:
        x, y = a[k], b[k]
        assert x.shape == y.shape, k
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), k
    for k in ["eps", "K_eps", "X0", "invX0", "eps_cvx", "del_ccv", "K_cvx", "K_ccv"]:
        assert a[k] == b[k], k


@pytest.mark.parametrize("dist", [0, 1])
@pytest.mark.parametrize("i_max", [8, 16, 32, 64, 128, 256])
def test_trad_tables_match_oracle(zig, O, dist, i_max):
    """Traditional stack (the comparison sampler of Table 1): the library's
    bisection on the top layer's area and the oracle's bisection on the
    closure f_{n-1} = 1 give the same doubles; the quick-accept thresholds
    are the integers below which k 2^-53 < k_i."""
    a = zig.zig_get_trad_tables(dist, i_max)
    b = O.trad_arrays(dist, i_max)
    assert a["n"] == b["n"] == i_max and a["b"] == b["b"]
    for k in ["X", "f", "W", "WS", "k"]:
        assert np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)), k
    for k in ["r", "v", "invr"]:
        assert a[k] == b[k], k
    kq = a["KQ"].astype(object)
    for i in range(i_max):
        ki = b["k"][i]
        q = int(kq[i])
        # the smallest integer q with q 2^-53 >= k_i
        assert q * 2.0 ** -53 >= ki and (q == 0 or (q - 1) * 2.0 ** -53 < ki), i


def test_bad_table_arguments(zig):
    for dist, i_max in [(2, 256), (0, 12), (0, 4), (1, 2048), (0, 0)]:
        with pytest.raises(zig.ZigError) as e:
            zig.zig_get_tables(dist, i_max)
        assert e.value.status == zig.ZIG_EINVAL
    for dist, i_max in [(2, 256), (0, 12), (0, 4), (1, 512), (0, 1024), (0, 0)]:
        with pytest.raises(zig.ZigError) as e:
            zig.zig_get_trad_tables(dist, i_max)
        assert e.value.status == zig.ZIG_EINVAL
    with pytest.raises(zig.ZigError):
        zig.zig_build_tables(100)


def test_fill_argument_validation(zig):
    """Invalid arguments fail with ZIG_EINVAL and a message, before any
    device work; n = 0 is a no-op."""
    fake = 1 << 20  # never dereferenced: every call below fails validation
    bad = [
        lambda: zig.zig_fill_exp(1, 0, 10, 0, 0.0, fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, -1.0, fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, float("nan"), fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, float("inf"), fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, 5e-324, fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 2, 1.0, fake),
        lambda: zig.zig_fill_normal(1, 0, 10, 0, 0.0, 0.0, fake),
        lambda: zig.zig_fill_normal(1, 0, 10, 0, float("nan"), 1.0, fake),
        lambda: zig.zig_fill_normal(1, 0, 10, 0, 0.0, float("inf"), fake),
        lambda: zig.zig_fill_normal(1, 0, 10, 1, 0.0, -2.0, fake),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, 1.0, None),
        lambda: zig.zig_fill_exp(1, 0, 10, 0, 1.0, fake + 4),
        lambda: zig.zig_fill_exp(1, 0, 10, 1, 1.0, fake + 2),
        lambda: zig.zig_fill_exp(1, 2 ** 64 - 5, 6, 0, 1.0, fake),
        lambda: zig.zig_fill(3, 0, 1, 0, 10, 1.0, 1.0, fake),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"i_max": 100}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"wg": 96}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"wg": 512, "spl": 8}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"wg": 128, "spl": 10}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"wg": 256, "spl": 12}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"flags": 4}),
        # the traditional sampler: FP64 only, no trace, not with the accelerated variant, no moments
        lambda: zig.zig_fill(0, 1, 1, 0, 10, 1.0, 1.0, fake, launch={"flags": zig.LAUNCH_TRADITIONAL}),
        lambda: zig.zig_fill(1, 0, 1, 0, 10, 0.0, 1.0, fake, launch={"flags": 3}),
        lambda: zig.zig_fill_trace(0, 0, 1, 0, 10, 1.0, 1.0, fake, fake, fake, fake, fake,
                                   launch={"flags": zig.LAUNCH_TRADITIONAL}),
        lambda: zig.zig_moments(0, 0, 1, 0, 10, 1.0, 1.0, fake, None, zig.Launch(0, 0, 0, zig.LAUNCH_TRADITIONAL)),
        # tables of more than 256 layers: plain fills only
        lambda: zig.zig_fill(1, 0, 1, 0, 10, 0.0, 1.0, fake, launch={"i_max": 1024, "flags": 1}),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"i_max": 512, "flags": zig.LAUNCH_TRADITIONAL}),
        lambda: zig.zig_moments(0, 0, 1, 0, 10, 1.0, 1.0, fake, None, zig.Launch(1024, 0, 0, 0)),
        lambda: zig.zig_fill(0, 0, 1, 0, 10, 1.0, 1.0, fake, launch={"i_max": 2048}),
    ]
    for k, f in enumerate(bad):
        with pytest.raises(zig.ZigError) as e:
            f()
        assert e.value.status == zig.ZIG_EINVAL, k
        assert zig.zig_last_error() != "", k
    # n = 0: no-op even with a null pointer
    zig.zig_fill_exp(1, 0, 0, 0, 1.0, None)
    zig.zig_fill_normal(1, 2 ** 64 - 1, 0, 1, 0.0, 1.0, None)
    assert zig.zig_last_error() == ""


def test_autotune_bad_flags_refused_before_device_work():
    from paper_1403_6870_amd import zig
    for flags in (4, 3):
        with pytest.raises(zig.ZigError) as e:
            zig.zig_autotune(None, flags)
        assert e.value.status == zig.ZIG_EINVAL


@pytest.mark.parametrize("i_max", [8, 256, 1024])
def test_normal_box_squeeze_agrees_with_density_test(zig, O, i_max):
    """The library's per-box squeeze of the plain normal box test decides
    points without evaluating the density: every point it calls accepted
    (k1 + k2 < sq_lo) the oracle's density test accepts, and every point it
    calls rejected (k1 + k2 >= sq_hi) the test rejects: probed along both
    boundaries and at random inside both regions, in every box."""
    t = zig.zig_get_tables(NORMAL, i_max)
    assert zig.zig_get_tables(EXP, i_max)["sq_lo"] is None
    L, X = t["L"], t["X"]
    lo, hi = t["sq_lo"].astype(object), t["sq_hi"].astype(object)
    one53, top = 2 ** 53, 2 ** 53 - 1
    rng = np.random.default_rng(i_max)
    decided = []

    def probe(total, want, j):
        a, b = max(0, total - top), min(total, top)
        if a > b:
            return
        ks = {a, b} | {int(v) for v in np.linspace(a, b, 33)} | {int(v) for v in rng.integers(a, b + 1, 16)}
        for k1 in ks:
            got, _ = O.box_attempt(NORMAL, i_max, j, k1, total - k1)
            assert got == want, (j, k1, total - k1, want)

    for j in range(1, L + 1):
        convex, concave = X[j] >= 1.0, X[j - 1] <= 1.0
        if convex:
            assert hi[j] == one53 + 2 ** 33 and lo[j] < one53
        elif concave:
            assert lo[j] == one53 - 2 ** 33 and hi[j] > one53
        else:
            assert lo[j] == 0 and hi[j] == 2 ** 55
            continue
        probe(lo[j] - 1, True, j)
        probe(hi[j], False, j)
        for _ in range(8):
            probe(int(rng.integers(0, lo[j])), True, j)
            probe(int(rng.integers(hi[j], 2 * top + 1)), False, j)
        # share of the box the squeeze decides (area under u + v = s is s^2 / 2)
        s_lo, s_hi = lo[j] / one53, hi[j] / one53
        decided.append(s_lo * s_lo / 2 + (2 - s_hi) ** 2 / 2)
    assert np.mean(decided) > 0.8
