"""zig_moments_noalloc (the entry point that allocates nothing, for
callers under graph capture or in serving loops) against zig_moments: two
calls in a row, the second smaller, give the same sums bit for bit (same
kernels, same workgroup count, same order) and lie within the rounding
bound of the oracle's exact sums; a call captured into a graph replays
correctly; missing tables are refused."""
import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    zig.zig_build_tables(256)
    return torch, zig


def noalloc(zig, torch, dist, dtype, seed, first, n, p0, p1, stream=None):
    s = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    st = (stream or torch.cuda.current_stream()).cuda_stream
    zig.zig_moments_noalloc(dist, dtype, seed, first, n, p0, p1, s.data_ptr(), st)
    return s


def within_bound(got, want, wabs, dtype, first, n, spl=32):
    per = 2 if dtype == F64 else 4
    blocks = (first + n - 1) // per - first // per + 1
    tiles = -(-blocks // (256 * spl))
    h = 2 * spl * per * -(-tiles // min(tiles, 256)) + -(-min(tiles, 4096) // 256) + 18
    gamma = h * U / (1 - h * U)
    for p in range(5):
        assert abs(got[p] - want[p]) <= (gamma + 2 * U) * wabs[p] + 1e-300, p


@pytest.mark.parametrize("dist,dtype", [(EXP, F64), (NORMAL, F64), (NORMAL, F32)])
def test_noalloc_equals_moments_twice(O, env, dist, dtype):
    torch, zig = env
    p0, p1 = (2.5, 0.0) if dist == EXP else (-1.0, 3.0)
    scale, shift = (1.0 / p0, 0.0) if dist == EXP else (p1, p0)
    for seed, first, n in [(11, 3, 20_000_011), (12, 7, 333_333)]:  # the second call is smaller
        got = noalloc(zig, torch, dist, dtype, seed, first, n, p0, p1).cpu().numpy()
        ref = zig.moments(dist, dtype, n, seed, first, p0, p1).cpu().numpy()
        assert got.tobytes() == ref.tobytes(), (seed, n)
        want, wabs = O.moments(dist, dtype, seed, first, n, scale, shift, threads=16, with_abs=True)
        within_bound(got, want, wabs, dtype, first, n)


def test_noalloc_captured_and_replayed(env):
    torch, zig = env
    n = 5_000_003
    ref = zig.moments(NORMAL, F64, n, 21, 1, 0.5, 2.0).cpu().numpy()
    s = torch.zeros(5, dtype=torch.float64, device="cuda")
    cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cap):
        zig.zig_moments_noalloc(NORMAL, F64, 21, 1, n, 0.5, 2.0, s.data_ptr(), cap.cuda_stream)
    for _ in range(3):
        s.fill_(float("nan"))
        other = zig.moments(EXP, F64, 1_000_000, 5, 0, 1.0, 0.0)  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert s.cpu().numpy().tobytes() == ref.tobytes()
        assert np.isfinite(other.cpu().numpy()).all()


def test_noalloc_refuses_missing_tables_and_bad_arguments(env):
    torch, zig = env
    s = torch.empty(5, dtype=torch.float64, device="cuda")
    with pytest.raises(zig.ZigError) as e:  # no GPU test builds 64-layer tables
        zig.zig_moments_noalloc(EXP, F64, 1, 0, 100, 1.0, 0.0, s.data_ptr(), None, zig.Launch(64, 0, 0, 0))
    assert e.value.status == zig.ZIG_ESTATE
    with pytest.raises(zig.ZigError) as e:
        zig.zig_moments_noalloc(EXP, F64, 1, 0, 100, -1.0, 0.0, s.data_ptr())
    assert e.value.status == zig.ZIG_EINVAL
    z = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    zig.zig_moments_noalloc(EXP, F64, 1, 0, 0, 1.0, 0.0, z.data_ptr())
    assert z.cpu().numpy().tolist() == [0.0] * 5
