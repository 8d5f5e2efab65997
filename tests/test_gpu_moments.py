"""GPU parity of the fused generate-and-reduce (zig_moments): the five raw
moment sums are bit-identical to the oracle's, which adds in the same fixed
order, for both distributions and output types, ragged and offset ranges,
ranges of one and zero outputs, small tables, and a range spanning two
segments of the device reduction; and they equal the moments of the fill's
own output (the same samples)."""
import math

import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


def params(dist, p0, p1):
    return (1.0 / p0, 0.0) if dist == EXP else (p1, p0)


@pytest.mark.parametrize("dist,dtype,seed,first,n,p0,p1", [
    (EXP, F64, 1, 0, 1_000_000, 1.0, 0.0),
    (NORMAL, F64, 7, 3, 3 * 2 ** 20 + 5, 0.0, 1.0),
    (EXP, F32, 11, 1, 777_777, 2.5, 0.0),
    (NORMAL, F32, 12, 2 ** 40 + 2, 2 ** 22 + 3, -1.0, 3.0),
    (EXP, F64, 5, 2 ** 64 - 1000, 1000, 0.7, 0.0),
    (NORMAL, F64, 5, 9, 1, 0.0, 1.0),
])
def test_moments_bit_identical_to_oracle(O, env, dist, dtype, seed, first, n, p0, p1):
    torch, zig = env
    got = zig.moments(dist, dtype, n, seed, first, p0, p1).cpu().numpy()
    scale, shift = params(dist, p0, p1)
    want = O.moments(dist, dtype, seed, first, n, scale, shift, threads=16)
    assert got.tobytes() == want.tobytes(), (got, want)


def test_moments_two_segments(O, env):
    """2^28 + 4101 FP64 outputs from an odd first index: more than one
    segment of 2^16 tiles."""
    torch, zig = env
    n = 2 ** 28 + 4101
    got = zig.moments(NORMAL, F64, n, 21, 5, 0.5, 2.0).cpu().numpy()
    want = O.moments(NORMAL, F64, 21, 5, n, 2.0, 0.5, threads=16)
    assert got.tobytes() == want.tobytes(), (got, want)


def test_moments_small_table_and_empty(O, env):
    torch, zig = env
    got = zig.moments(EXP, F64, 100_003, 3, 0, 1.5, 0.0, i_max=8).cpu().numpy()
    want = O.moments(EXP, F64, 3, 0, 100_003, 1.0 / 1.5, 0.0, threads=8, i_max=8)
    assert got.tobytes() == want.tobytes()
    z = zig.moments(EXP, F64, 0, 3, 0, 1.5, 0.0).cpu().numpy()
    assert z.tolist() == [0.0] * 5


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
    for p in range(5):
        exact = math.fsum(q[p])
        assert abs(got[p] - exact) <= 1e-12 * math.fsum(np.abs(q[p])), p


def test_moments_reject_bad_arguments(env):
    torch, zig = env
    s = torch.empty(5, dtype=torch.float64, device="cuda")
    for args in [(2, F64, 1, 0, 10, 1.0, 0.0), (EXP, 3, 1, 0, 10, 1.0, 0.0), (EXP, F64, 1, 0, 10, -1.0, 0.0),
                 (NORMAL, F64, 1, 0, 10, 0.0, 0.0), (EXP, F64, 1, 2 ** 64 - 5, 10, 1.0, 0.0)]:
        with pytest.raises(zig.ZigError) as e:
            zig.zig_moments(*args, s.data_ptr())
        assert e.value.status == zig.ZIG_EINVAL
    with pytest.raises(zig.ZigError):
        zig.zig_moments(EXP, F64, 1, 0, 10, 1.0, 0.0, s.data_ptr(), None, zig.Launch(256, 512, 4))
