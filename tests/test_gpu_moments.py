"""GPU parity of the fused generate-and-reduce (zig_moments).

The oracle's sums are the exact sums of the powers rounded once; the GPU
adds in its own order, so each GPU sum must lie within the rounding bound
that zig.h states for that order, (gamma_h + 2u) sum |x^p|, around the
oracle's value (one u for the fused multiply-adds of the odd powers, one
for the oracle's own final rounding).  A dropped, doubled or wrong output
moves a sum by about 1/n of sum |x| or more, far outside the bound at
these sizes.  Covered: both distributions and output types, ragged and
offset ranges, ranges of one and zero outputs, small tables, the
accelerated normal variant, all tile shapes, a range of 2^28 outputs, the
moments of the fill's own output, determinism, and argument checks."""
import math

import ctypes

import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
MAX_GROUPS = 4096  # the most workgroups one launch uses
MIN_GROUPS = 256   # it uses at least min(tiles, 256) (one per compute unit)


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


def params(dist, p0, p1):
    return (1.0 / p0, 0.0) if dist == EXP else (p1, p0)


def depth(dtype, first, n, spl=32):
    """The longest chain of additions zig.h allows for these arguments."""
    per = 2 if dtype == F64 else 4
    blocks = (first + n - 1) // per - first // per + 1
    tiles = -(-blocks // (256 * spl))
    g_min = min(tiles, MIN_GROUPS)
    g_max = min(tiles, MAX_GROUPS)
    return 2 * spl * per * -(-tiles // g_min) + 6 + 4 + -(-g_max // 256) + 8


def check(got, want, wabs, h):
    gamma = h * U / (1 - h * U)
    for p in range(5):
        bound = (gamma + 2 * U) * wabs[p] + 1e-300
        assert abs(got[p] - want[p]) <= bound, (p, got[p], want[p], bound)


CASES = [
    (EXP, F64, 1, 0, 1_000_000, 1.0, 0.0),
    (NORMAL, F64, 7, 3, 3 * 2 ** 20 + 5, 0.0, 1.0),
    (EXP, F32, 11, 1, 777_777, 2.5, 0.0),
    (NORMAL, F32, 12, 2 ** 40 + 2, 2 ** 22 + 3, -1.0, 3.0),
    (EXP, F64, 5, 2 ** 64 - 1000, 1000, 0.7, 0.0),
    (NORMAL, F64, 5, 9, 1, 0.0, 1.0),
    (NORMAL, F32, 3, 7, 5, 2.0, 0.5),
]


@pytest.mark.parametrize("dist,dtype,seed,first,n,p0,p1", CASES)
def test_moments_match_oracle(O, env, dist, dtype, seed, first, n, p0, p1):
    torch, zig = env
    got = zig.moments(dist, dtype, n, seed, first, p0, p1).cpu().numpy()
    scale, shift = params(dist, p0, p1)
    want, wabs = O.moments(dist, dtype, seed, first, n, scale, shift, threads=16, with_abs=True)
    check(got, want, wabs, depth(dtype, first, n))


@pytest.mark.parametrize("spl", [16, 32, 64])
@pytest.mark.parametrize("dist,dtype", [(EXP, F64), (NORMAL, F64), (EXP, F32), (NORMAL, F32)])
def test_moments_every_shape(O, env, spl, dist, dtype):
    torch, zig = env
    n, first, seed, p0, p1 = 2_345_679, 13, 99, (1.5 if dist == EXP else -0.5), 2.0
    got = zig.moments(dist, dtype, n, seed, first, p0, p1, spl=spl).cpu().numpy()
    scale, shift = params(dist, p0, p1)
    want, wabs = O.moments(dist, dtype, seed, first, n, scale, shift, threads=16, with_abs=True)
    check(got, want, wabs, depth(dtype, first, n, spl))


def test_moments_accelerated_variant(O, env):
    torch, zig = env
    n = 1_234_567
    got = zig.moments(NORMAL, F64, n, 4, 2, 0.25, 1.5, accel=True).cpu().numpy()
    want, wabs = O.moments(NORMAL, F64, 4, 2, n, 1.5, 0.25, threads=16, accel=True, with_abs=True)
    check(got, want, wabs, depth(F64, 2, n))


def test_moments_2_28(O, env):
    """2^28 + 4101 FP64 outputs from an odd first index."""
    torch, zig = env
    n = 2 ** 28 + 4101
    got = zig.moments(NORMAL, F64, n, 21, 5, 0.5, 2.0).cpu().numpy()
    want, wabs = O.moments(NORMAL, F64, 21, 5, n, 2.0, 0.5, threads=16, with_abs=True)
    check(got, want, wabs, depth(F64, 5, n))


def test_moments_small_table_and_empty(O, env):
    torch, zig = env
    got = zig.moments(EXP, F64, 100_003, 3, 0, 1.5, 0.0, i_max=8).cpu().numpy()
    want, wabs = O.moments(EXP, F64, 3, 0, 100_003, 1.0 / 1.5, 0.0, threads=8, i_max=8, with_abs=True)
    check(got, want, wabs, depth(F64, 0, 100_003))
    z = zig.moments(EXP, F64, 0, 3, 0, 1.5, 0.0).cpu().numpy()
    assert z.tolist() == [0.0] * 5


def test_moments_deterministic(env):
    torch, zig = env
    a = zig.moments(NORMAL, F64, 50_000_017, 8, 3, 1.0, 2.0).cpu().numpy()
    b = zig.moments(NORMAL, F64, 50_000_017, 8, 3, 1.0, 2.0).cpu().numpy()
    assert a.tobytes() == b.tobytes()


def test_moments_match_fill_output(env):
    torch, zig = env
    n = 5_000_011
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    zig.fill(x, NORMAL, 33, 17, 1.0, 2.0)
    got = zig.moments(NORMAL, F32, n, 33, 17, 1.0, 2.0).cpu().numpy()
    d = x.cpu().numpy().astype(np.float64)
    q = [d, d * d]
    q += [q[1] * d, q[1] * q[1]]
    q += [q[3] * d]
    h = depth(F32, 17, n)
    for p in range(5):
        exact = math.fsum(q[p])
        assert abs(got[p] - exact) <= (h * U / (1 - h * U) + 2 * U) * math.fsum(np.abs(q[p])), p


def test_moments_reject_bad_arguments(env):
    torch, zig = env
    s = torch.empty(5, dtype=torch.float64, device="cuda")
    for args in [(2, F64, 1, 0, 10, 1.0, 0.0), (EXP, 3, 1, 0, 10, 1.0, 0.0), (EXP, F64, 1, 0, 10, -1.0, 0.0),
                 (NORMAL, F64, 1, 0, 10, 0.0, 0.0), (EXP, F64, 1, 2 ** 64 - 5, 10, 1.0, 0.0)]:
        with pytest.raises(zig.ZigError) as e:
            zig.zig_moments(*args, s.data_ptr())
        assert e.value.status == zig.ZIG_EINVAL
    for la in [zig.Launch(256, 512, 4), zig.Launch(256, 256, 7), zig.Launch(512, 0, 0, 0)]:
        with pytest.raises(zig.ZigError) as e:
            zig.zig_moments(EXP, F64, 1, 0, 10, 1.0, 0.0, s.data_ptr(), None, la)
        assert e.value.status == zig.ZIG_EINVAL


def test_moments_per_thread_stream_and_capture(env):
    """The per-thread stream handle is accepted (each launch has its own
    scratch slot) and gives the same bits; a capturing stream is refused
    before any work, since a graph would fix the scratch slot."""
    torch, zig = env
    s = torch.empty(5, dtype=torch.float64, device="cuda")
    zig.zig_moments(NORMAL, F64, 9, 3, 3_000_001, 1.0, 2.0, s.data_ptr(), 2)  # hipStreamPerThread
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    assert hip.hipStreamSynchronize(ctypes.c_void_p(2)) == 0
    ref = zig.moments(NORMAL, F64, 3_000_001, 9, 3, 1.0, 2.0).cpu().numpy()
    assert s.cpu().numpy().tobytes() == ref.tobytes()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        g = torch.cuda.CUDAGraph()
        g.capture_begin()
        try:
            with pytest.raises(zig.ZigError) as e:
                zig.zig_moments(EXP, F64, 1, 0, 10, 1.0, 0.0, s.data_ptr(), side.cuda_stream)
            assert e.value.status == zig.ZIG_EINVAL
            s.zero_()
        finally:
            g.capture_end()
    torch.cuda.synchronize()
