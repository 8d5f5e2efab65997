"""ctypes wrapper around the scalar CPU oracle (zig_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle is the reference the GPU library is
checked against; only the tests, the smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the library.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzig_oracle.so")
SRC = os.path.join(HERE, "zig_oracle.c")

EXP, NORMAL = 0, 1
F64, F32 = 0, 1
MAXI = 1024


def build(force=False):
    """Compile the oracle with gcc: IEEE round-to-nearest, no contraction,
    no fast-math, so that only the explicit fma calls are fused."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           SRC, "-o", tmp, "-lquadmath", "-lm", "-lpthread"]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


class Trad(ctypes.Structure):
    _fields_ = [
        ("dist", ctypes.c_int), ("n", ctypes.c_uint32), ("b", ctypes.c_uint32),
        ("X", ctypes.c_double * (MAXI + 1)), ("f", ctypes.c_double * (MAXI + 1)),
        ("W", ctypes.c_double * MAXI), ("WS", ctypes.c_double * MAXI), ("k", ctypes.c_double * MAXI),
        ("v", ctypes.c_double), ("r", ctypes.c_double), ("invr", ctypes.c_double),
        ("hp_r", ctypes.c_char * 48), ("hp_v", ctypes.c_char * 48),
    ]


class Tables(ctypes.Structure):
    _fields_ = [
        ("dist", ctypes.c_int), ("i_max", ctypes.c_uint32), ("b", ctypes.c_uint32), ("L", ctypes.c_uint32),
        ("X", ctypes.c_double * (MAXI + 1)), ("f", ctypes.c_double * (MAXI + 1)),
        ("XS", ctypes.c_double * MAXI), ("XS32", ctypes.c_float * MAXI),
        ("W", ctypes.c_double * (MAXI + 1)), ("H", ctypes.c_double * (MAXI + 1)),
        ("q", ctypes.c_uint64 * (MAXI + 1)), ("T", ctypes.c_uint64 * MAXI), ("A", ctypes.c_uint32 * MAXI),
        ("eps", ctypes.c_double), ("K_eps", ctypes.c_uint64), ("X0", ctypes.c_double), ("invX0", ctypes.c_double),
        ("eps_cvx", ctypes.c_double), ("del_ccv", ctypes.c_double), ("K_cvx", ctypes.c_uint64),
        ("K_ccv", ctypes.c_uint64), ("accel", ctypes.c_int),
        ("hpX", (ctypes.c_char * 48) * (MAXI + 1)), ("hpf", (ctypes.c_char * 48) * (MAXI + 1)),
        ("hpA", (ctypes.c_char * 48) * (MAXI + 1)),
        ("hp_area", ctypes.c_char * 48), ("hp_total", ctypes.c_char * 48), ("hp_eps", ctypes.c_char * 48),
        ("hp_eps_cvx", ctypes.c_char * 48), ("hp_del_ccv", ctypes.c_char * 48),
    ]


_lib = None
_tables = {}


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        u64, u32, i32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        tp = ctypes.POINTER(Tables)
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.orc_philox4x32_10.restype = None
        L.orc_build_tables.argtypes = [i32, u32, tp]
        L.orc_build_tables.restype = i32
        L.orc_fill.argtypes = [i32, i32, tp, tp, u64, u64, u64, dbl, dbl, vp, i32]
        L.orc_fill.restype = i32
        L.orc_fill_trace.argtypes = [i32, i32, tp, tp, u64, u64, u64, dbl, dbl, vp, vp, vp, vp, vp]
        L.orc_fill_trace.restype = i32
        L.orc_box_attempt.argtypes = [tp, u32, u64, u64, ctypes.POINTER(dbl)]
        L.orc_box_attempt.restype = i32
        L.orc_box_grid.argtypes = [tp, u32, u32, u32, vp, vp]
        L.orc_box_grid.restype = i32
        L.orc_sample_region.argtypes = [tp, tp, i32, u32, u64, u64, u64, vp]
        L.orc_sample_region.restype = i32
        L.orc_alias_draw.argtypes = [tp, u64]
        L.orc_alias_draw.restype = u32
        L.orc_moments.argtypes = [i32, i32, tp, tp, u64, u64, u64, dbl, dbl, ctypes.POINTER(dbl),
                                  ctypes.POINTER(dbl), i32]
        L.orc_moments.restype = i32
        L.orc_exact_sum.argtypes = [vp, u64, ctypes.POINTER(dbl)]
        L.orc_exact_sum.restype = i32
        trp = ctypes.POINTER(Trad)
        L.orc_build_trad.argtypes = [i32, u32, trp]
        L.orc_build_trad.restype = i32
        L.orc_trad_fill.argtypes = [i32, trp, trp, u64, u64, u64, dbl, dbl, vp, vp, i32]
        L.orc_trad_fill.restype = i32
        L.orc_trad_size.argtypes = []
        L.orc_trad_size.restype = u64
        if L.orc_trad_size() != ctypes.sizeof(Trad):
            raise RuntimeError("oracle traditional table layout mismatch")
        L.orc_tables_size.argtypes = []
        L.orc_tables_size.restype = u64
        if L.orc_tables_size() != ctypes.sizeof(Tables):
            raise RuntimeError("oracle table layout mismatch")
        _lib = L
    return _lib


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def tables(dist, i_max=256, accel=False):
    """Tables of `dist`; accel=True gives the normal tables that select the
    accelerated overhang variant."""
    key = (dist, i_max, bool(accel) and dist == NORMAL)
    if key not in _tables:
        t = Tables()
        if lib().orc_build_tables(dist, i_max, ctypes.byref(t)) != 0:
            raise ValueError("unsupported table %r" % (key,))
        t.accel = 1 if key[2] else 0
        _tables[key] = t
    return _tables[key]


_trad = {}


def trad(dist, n=256):
    """Traditional-ziggurat tables of `dist` with n layers."""
    key = (dist, n)
    if key not in _trad:
        t = Trad()
        if lib().orc_build_trad(dist, n, ctypes.byref(t)) != 0:
            raise ValueError("unsupported traditional table %r" % (key,))
        _trad[key] = t
    return _trad[key]


def trad_arrays(dist, n=256):
    t = trad(dist, n)
    return {"n": t.n, "b": t.b, "X": np.array(t.X[:n]), "f": np.array(t.f[:n]), "W": np.array(t.W[:n]),
            "WS": np.array(t.WS[:n]), "k": np.array(t.k[:n]), "v": t.v, "r": t.r, "invr": t.invr,
            "hp_r": t.hp_r.decode(), "hp_v": t.hp_v.decode()}


def trad_fill(dist, seed, first, n, scale, shift=0.0, threads=1, layers=256, words=False):
    """FP64 outputs of the traditional sampler (and the slow words used per
    output if words=True)."""
    out = np.empty(n, dtype=np.float64)
    w = np.empty(n, dtype=np.uint32) if words else None
    ex = ctypes.byref(trad(EXP, layers))
    nt = ctypes.byref(trad(NORMAL, layers)) if dist == NORMAL else None
    r = lib().orc_trad_fill(dist, ex, nt, seed, first, n, scale, shift, out.ctypes.data if n else None,
                            w.ctypes.data if words and n else None, threads)
    if r != 0:
        raise ValueError("orc_trad_fill rejected its arguments")
    return (out, w) if words else out


def table_arrays(dist, i_max=256):
    """The tables as numpy arrays (copies)."""
    t = tables(dist, i_max)
    L = t.L
    return {
        "L": L, "i_max": t.i_max, "b": t.b,
        "X": np.array(t.X[: L + 1]), "f": np.array(t.f[: L + 1]),
        "XS": np.array(t.XS[: t.i_max]), "XS32": np.array(t.XS32[: t.i_max], dtype=np.float32),
        "W": np.array(t.W[: L + 1]), "H": np.array(t.H[: L + 1]),
        "q": np.array(t.q[: L + 1], dtype=np.uint64),
        "T": np.array(t.T[: t.i_max], dtype=np.uint64), "A": np.array(t.A[: t.i_max], dtype=np.uint32),
        "eps": t.eps, "K_eps": int(t.K_eps), "X0": t.X0, "invX0": t.invX0,
        "hpX": [t.hpX[k].value.decode() for k in range(L + 1)],
        "hpf": [t.hpf[k].value.decode() for k in range(L + 1)],
        "hpA": [t.hpA[k].value.decode() for k in range(L + 1)],
        "hp_area": t.hp_area.decode(), "hp_total": t.hp_total.decode(),
        "hp_eps": t.hp_eps.decode(),
        "eps_cvx": t.eps_cvx, "del_ccv": t.del_ccv, "K_cvx": int(t.K_cvx), "K_ccv": int(t.K_ccv),
        "hp_eps_cvx": t.hp_eps_cvx.decode(), "hp_del_ccv": t.hp_del_ccv.decode(),
    }


def _tabs(dist, i_max, accel=False):
    ex = tables(EXP, i_max)
    nt = tables(NORMAL, i_max, accel) if dist == NORMAL else None
    return ctypes.byref(ex), (ctypes.byref(nt) if nt is not None else None)


def fill(dist, dtype, seed, first, n, scale, shift=0.0, threads=1, i_max=256, accel=False):
    out = np.empty(n, dtype=np.float64 if dtype == F64 else np.float32)
    ex, nt = _tabs(dist, i_max, accel)
    r = lib().orc_fill(dist, dtype, ex, nt, seed, first, n, scale, shift,
                       out.ctypes.data if n else None, threads)
    if r != 0:
        raise ValueError("orc_fill rejected its arguments")
    return out


def moments(dist, dtype, seed, first, n, scale, shift=0.0, threads=1, i_max=256, accel=False, with_abs=False):
    """Raw moment sums (S1..S5) of the outputs of the same fill, each the
    exact sum rounded once; with_abs=True also returns the sums of |x^p|."""
    out = (ctypes.c_double * 5)()
    absd = (ctypes.c_double * 5)()
    ex, nt = _tabs(dist, i_max, accel)
    if lib().orc_moments(dist, dtype, ex, nt, seed, first, n, scale, shift, out, absd, threads) != 0:
        raise ValueError("orc_moments rejected its arguments")
    s = np.array(list(out))
    return (s, np.array(list(absd))) if with_abs else s


def exact_sum(x):
    """The exact sum of the doubles in x, rounded once to double."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    s = ctypes.c_double()
    if lib().orc_exact_sum(a.ctypes.data if a.size else None, a.size, ctypes.byref(s)) != 0:
        raise ValueError("orc_exact_sum rejected its arguments")
    return s.value


def fill_trace(dist, dtype, seed, first, n, scale, shift=0.0, i_max=256, accel=False):
    out = np.empty(n, dtype=np.float64 if dtype == F64 else np.float32)
    layer = np.empty(n, dtype=np.uint32)
    region = np.empty(n, dtype=np.int32)
    words = np.empty(n, dtype=np.uint32)
    tests = np.empty(n, dtype=np.uint32)
    ex, nt = _tabs(dist, i_max, accel)
    r = lib().orc_fill_trace(dist, dtype, ex, nt, seed, first, n, scale, shift,
                             out.ctypes.data, layer.ctypes.data, region.ctypes.data,
                             words.ctypes.data, tests.ctypes.data)
    if r != 0:
        raise ValueError("orc_fill_trace rejected its arguments")
    return out, layer, region, words, tests


def box_attempt(dist, i_max, j, k1, k2, accel=False):
    x = ctypes.c_double()
    r = lib().orc_box_attempt(ctypes.byref(tables(dist, i_max, accel)), j, k1, k2, ctypes.byref(x))
    if r < 0:
        raise ValueError("bad box attempt")
    return bool(r), x.value


def box_grid(dist, i_max, j, g, shift, accel=False):
    """Attempts of box j over the g x g lattice (a << shift, c << shift)."""
    acc = np.empty(g * g, dtype=np.uint8)
    x = np.empty(g * g, dtype=np.float64)
    r = lib().orc_box_grid(ctypes.byref(tables(dist, i_max, accel)), j, g, shift, acc.ctypes.data,
                           x.ctypes.data)
    if r != 0:
        raise ValueError("bad box grid")
    return acc.reshape(g, g).astype(bool), x.reshape(g, g)


def sample_region(dist, j, seed, index0, n, i_max=256, accel=False):
    out = np.empty(n, dtype=np.float64)
    ex, nt = _tabs(dist, i_max, accel)
    r = lib().orc_sample_region(ex, nt, dist, j, seed, index0, n, out.ctypes.data)
    if r != 0:
        raise ValueError("bad region")
    return out


def alias_draw(dist, i_max, r):
    return int(lib().orc_alias_draw(ctypes.byref(tables(dist, i_max)), r))
