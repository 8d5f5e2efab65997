"""GPU parity of the accelerated normal-overhang variant
(ZIG_LAUNCH_NORMAL_ACCEL): per-output trace parity with the oracle's
variant (layer, first region, slow-stream words, density evaluations and
values), full fills in both output types at several table sizes and
launch shapes, 2^30 fills element by element, and the exponential
ignoring the flag (the fused moments
with the variant are covered with the other moments tests)."""
import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL, parity, to_np

pytestmark = pytest.mark.gpu

ACCEL = 1


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


@pytest.mark.parametrize("i_max", [8, 256])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_trace_parity(O, env, dtype, i_max):
    torch, zig = env
    n = (1 << 18) + 77
    first = 1 << 33
    out = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    out, layer, region, words, tests = zig.fill_trace(out, NORMAL, 5, first, 0.0, 1.0,
                                                      launch={"i_max": i_max, "flags": ACCEL})
    w_out, w_layer, w_region, w_words, w_tests = O.fill_trace(NORMAL, dtype, 5, first, n, 1.0, 0.0, i_max=i_max,
                                                               accel=True)
    assert np.array_equal(to_np(layer).view(np.uint32), w_layer)
    assert np.array_equal(to_np(region), w_region)
    assert np.array_equal(to_np(words).view(np.uint32), w_words)
    assert np.array_equal(to_np(tests).view(np.uint32), w_tests)
    parity(to_np(out), w_out, 4 if dtype == F64 else 2)


@pytest.mark.parametrize("dtype,i_max,wg,spl", [(F64, 256, 0, 0), (F32, 256, 0, 0), (F64, 16, 128, 8),
                                                (F32, 8, 512, 2), (F64, 256, 64, 1)])
def test_fill_parity(O, env, dtype, i_max, wg, spl):
    torch, zig = env
    n = (1 << 22) + 13
    out = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    zig.fill(out, NORMAL, 31, 7, -1.0, 3.0, launch={"i_max": i_max, "wg": wg, "spl": spl, "flags": ACCEL})
    want = O.fill(NORMAL, dtype, 31, 7, n, 3.0, -1.0, threads=16, i_max=i_max, accel=True)
    got = to_np(out)
    it = np.int64 if dtype == F64 else np.int32
    assert np.array_equal(got.view(it), want.view(it))
    # the fast-path outputs are those of the default sampler
    plain = torch.empty_like(out)
    zig.fill(plain, NORMAL, 31, 7, -1.0, 3.0, launch={"i_max": i_max})
    same = (to_np(plain).view(it) == got.view(it)).mean()
    assert 0.95 < same < 1.0


@pytest.mark.slow
@pytest.mark.parametrize("dtype", [F64, F32])
def test_full_size_full_parity(O, env, dtype):
    """N(-1, 3), 2^30 outputs with the variant at the default shape (the
    configuration the benchmark times in FP64), every output against the
    oracle's variant in chunks of 2^26: bit-identical."""
    torch, zig = env
    n = 1 << 30
    out = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    zig.fill(out, NORMAL, 12, 0, -1.0, 3.0, launch={"flags": ACCEL})
    torch.cuda.synchronize()
    it = np.int64 if dtype == F64 else np.int32
    chunk = 1 << 26
    bad = 0
    for s in range(0, n, chunk):
        want = O.fill(NORMAL, dtype, 12, s, chunk, 3.0, -1.0, threads=16, accel=True)
        bad += int(np.count_nonzero(out[s:s + chunk].cpu().numpy().view(it) != want.view(it)))
    print("accel full t%d: %d outputs differ" % (dtype, bad), flush=True)
    assert bad == 0
    del out
    torch.cuda.empty_cache()


def test_exponential_ignores_flag(env):
    torch, zig = env
    n = 1 << 20
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    zig.fill(a, EXP, 3, 0, 1.5, 0.0)
    zig.fill(b, EXP, 3, 0, 1.5, 0.0, launch={"flags": ACCEL})
    assert torch.equal(a, b)


def test_unknown_flags_refused(env):
    torch, zig = env
    a = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(zig.ZigError) as e:
        zig.fill(a, NORMAL, 3, 0, 0.0, 1.0, launch={"flags": 6})
    assert e.value.status == zig.ZIG_EINVAL
