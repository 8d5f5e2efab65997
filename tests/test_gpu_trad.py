"""GPU parity of the traditional ziggurat (ZIG_LAUNCH_TRADITIONAL, the
comparison sampler of Table 1) against the oracle's traditional sampler,
through the C ABI.

Bar: bit-identical FP64 outputs.  Every output value is a product, a sum
or an fma of table entries and lattice values that both sides compute in
the same order; the density evaluations only decide accept or reject, so
any decision that differed would show as a different output."""
import numpy as np
import pytest

from helpers import EXP, NORMAL, to_np

pytestmark = pytest.mark.gpu

TRAD = 2


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


def _oracle(O, dist, seed, first, n, p0, p1, layers=256):
    if dist == EXP:
        return O.trad_fill(EXP, seed, first, n, 1.0 / p0, 0.0, threads=16, layers=layers)
    return O.trad_fill(NORMAL, seed, first, n, p1, p0, threads=16, layers=layers)


def _gpu(env, dist, seed, first, n, p0, p1, **launch):
    torch, zig = env
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    launch["flags"] = TRAD
    zig.fill(out, dist, seed, first, p0, p1, launch=launch)
    return out


def _same(got, want):
    diff = got.view(np.int64) != want.view(np.int64)
    nd = int(np.count_nonzero(diff))
    print("traditional: %d of %d outputs differ" % (nd, got.size), flush=True)
    assert nd == 0


@pytest.mark.parametrize("i_max", [8, 16, 256])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_parity_ragged(O, env, dist, i_max):
    """Several tiles plus a ragged tail, odd first index, non-trivial
    parameters; with 8 layers 27-37 % of the first draws miss the quick test."""
    n = (1 << 20) + 12345
    p0, p1 = (2.5, 0.0) if dist == EXP else (-1.0, 3.0)
    got = to_np(_gpu(env, dist, 11 + dist, 7, n, p0, p1, i_max=i_max))
    _same(got, _oracle(O, dist, 11 + dist, 7, n, p0, p1, layers=i_max))


@pytest.mark.parametrize("wg,spl", [(64, 1), (128, 8), (256, 8), (512, 4), (1024, 2)])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_parity_shapes(O, env, dist, wg, spl):
    """Forced launch shapes (every tile size the kernel is built for is
    covered by the smallest and largest here), large first index."""
    n = (1 << 19) + 3
    first = (1 << 40) + 1
    p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
    got = to_np(_gpu(env, dist, 5, first, n, p0, p1, wg=wg, spl=spl))
    _same(got, _oracle(O, dist, 5, first, n, p0, p1))


@pytest.mark.parametrize("n", [1, 2, 3, 63, 4097])
def test_tiny_and_edges(O, env, n):
    for dist in (EXP, NORMAL):
        p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
        got = to_np(_gpu(env, dist, 99, 2 ** 64 - n, n, p0, p1))
        _same(got, _oracle(O, dist, 99, 2 ** 64 - n, n, p0, p1))


@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_full_size_sampled(O, env, dist):
    """2^30 FP64 outputs in the launch configuration of the comparison
    (default shape), sampled chunks (head, tail, 16 random) against the
    oracle; mean and second moment of all outputs within 4.5 standard
    errors."""
    torch, zig = env
    n = 1 << 30
    seed = 11 if dist == EXP else 12
    p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
    out = _gpu(env, dist, seed, 0, n, p0, p1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    size = 1 << 14
    starts = [0, n - size] + sorted(int(v) for v in rng.integers(0, n - size, size=16))
    for s in starts:
        _same(out[s:s + size].cpu().numpy(), _oracle(O, dist, seed, s, size, p0, p1))
    m1 = float(out.mean())
    m2 = float((out * out).mean())
    if dist == EXP:
        assert abs(m1 - 1) < 4.5 / n ** 0.5
        assert abs(m2 - 2) < 4.5 * (20.0 / n) ** 0.5
    else:
        assert abs(m1) < 4.5 / n ** 0.5
        assert abs(m2 - 1) < 4.5 * (2.0 / n) ** 0.5
    del out
    torch.cuda.empty_cache()


@pytest.mark.slow
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_full_size_full_parity(O, env, dist):
    """The same 2^30 FP64 fills, every output against the oracle's
    traditional sampler in chunks of 2^26."""
    torch, zig = env
    n = 1 << 30
    seed = 11 if dist == EXP else 12
    p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
    out = _gpu(env, dist, seed, 0, n, p0, p1)
    torch.cuda.synchronize()
    chunk = 1 << 26
    for s in range(0, n, chunk):
        _same(out[s:s + chunk].cpu().numpy(), _oracle(O, dist, seed, s, chunk, p0, p1))
    del out
    torch.cuda.empty_cache()


def test_rejects_fp32_and_accel(env):
    torch, zig = env
    out = torch.empty(16, dtype=torch.float32, device="cuda")
    with pytest.raises(zig.ZigError) as e:
        zig.fill(out, EXP, 1, 0, 1.0, 0.0, launch={"flags": TRAD})
    assert e.value.status == zig.ZIG_EINVAL
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(zig.ZigError) as e:
        zig.fill(out, NORMAL, 1, 0, 0.0, 1.0, launch={"flags": TRAD | 1})
    assert e.value.status == zig.ZIG_EINVAL
