"""GPU parity of the fill kernels against the CPU oracle, through the C ABI.

Bar: FP64 outputs bit-identical on the fast path and within 4 ulp on the
slow paths with identical accept/reject decisions (the traces must match:
same layer, region, slow words and density evaluations per output); FP32
within 2 ulp.  All inputs are seeded.
"""
import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL, gpu_fill, oracle_fill, parity, to_np

pytestmark = pytest.mark.gpu

ULP = {F64: 4, F32: 2}
ZIG_LAUNCH_SHAPES = ([(w, s) for w in (64, 128, 256, 512, 1024) for s in (1, 2, 4, 8) if w * s <= 2048]
                     + [(256, 7), (256, 10)])


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _report(name, nd, mu):
    print("%s: %d outputs not bit-identical, max %d ulp" % (name, nd, mu), flush=True)


def test_c1_exp_1e6(O, torch_cuda):
    """Exponential rate 1, 10^6 FP64 samples, seed 1, 256 layers."""
    n = 10 ** 6
    got = to_np(gpu_fill(EXP, F64, 1, 0, n, 1.0, 0.0))
    want = oracle_fill(O, EXP, F64, 1, 0, n, 1.0, 0.0)
    nd, mu = parity(got, want, ULP[F64])
    _report("c1", nd, mu)
    assert nd == 0


@pytest.mark.parametrize("i_max", [8, 16, 256])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_parity_ragged(O, torch_cuda, dist, dtype, i_max):
    """Several tiles plus a ragged tail, odd first index, non-trivial
    parameters; small tables make the slow paths common."""
    n = (1 << 20) + 12345
    first = 7
    p0, p1 = (2.5, 0.0) if dist == EXP else (-1.0, 3.0)
    got = to_np(gpu_fill(dist, dtype, 11 + dist, first, n, p0, p1, launch={"i_max": i_max}))
    want = oracle_fill(O, dist, dtype, 11 + dist, first, n, p0, p1, i_max=i_max)
    scale, shift = (1.0 / p0, 0.0) if dist == EXP else (p1, p0)
    _, _, region, _, _ = O.fill_trace(dist, dtype, 11 + dist, first, n, scale, shift, i_max=i_max)
    nd, mu = parity(got, want, ULP[dtype], exact=region < 0)
    _report("ragged d%d t%d i%d" % (dist, dtype, i_max), nd, mu)


@pytest.mark.parametrize("i_max", [8, 256])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_trace_parity(O, torch_cuda, dist, dtype, i_max):
    """Stream counters and indices bit-exact: per output the same layer
    index, first region, number of slow-stream words and number of density
    evaluations as the oracle (so every accept/reject decision agrees)."""
    from paper_1403_6870_amd import zig
    torch = torch_cuda
    n = (1 << 18) + 77
    first = 1 << 33
    p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
    out = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    out, layer, region, words, tests = zig.fill_trace(out, dist, 5, first, p0, p1, launch={"i_max": i_max})
    got = to_np(out)
    if dist == EXP:
        w_out, w_layer, w_region, w_words, w_tests = O.fill_trace(dist, dtype, 5, first, n, 1.0 / p0, 0.0,
                                                                   i_max=i_max)
    else:
        w_out, w_layer, w_region, w_words, w_tests = O.fill_trace(dist, dtype, 5, first, n, p1, p0, i_max=i_max)
    assert np.array_equal(to_np(layer).view(np.uint32), w_layer)
    assert np.array_equal(to_np(region), w_region)
    assert np.array_equal(to_np(words).view(np.uint32), w_words)
    assert np.array_equal(to_np(tests).view(np.uint32), w_tests)
    nd, mu = parity(got, w_out, ULP[dtype], exact=w_region < 0)
    _report("trace d%d t%d i%d slow=%d" % (dist, dtype, i_max, int((w_region >= 0).sum())), nd, mu)


@pytest.mark.parametrize("i_max", [8, 256])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_launch_shape_independence(torch_cuda, dist, dtype, i_max):
    """Every compiled workgroup size x blocks-per-lane (tile and slow-queue
    depth) gives the same bits."""
    n = 3 * 512 * 8 * 4 + 1001
    p0, p1 = (0.7, 0.0) if dist == EXP else (0.5, 2.0)
    ref = to_np(gpu_fill(dist, dtype, 99, 3, n, p0, p1, launch={"i_max": i_max}))
    it = np.int64 if dtype == F64 else np.int32
    for wg, spl in ZIG_LAUNCH_SHAPES:
        launch = {"i_max": i_max, "wg": wg, "spl": spl}
        got = to_np(gpu_fill(dist, dtype, 99, 3, n, p0, p1, launch=launch))
        assert np.array_equal(got.view(it), ref.view(it)), (wg, spl)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_split_calls_concatenate(torch_cuda, dist, dtype):
    """fill(first, n) == fill(first, a) ++ fill(first + a, n - a)."""
    torch = torch_cuda
    n = 200003
    first = 12345
    whole = to_np(gpu_fill(dist, dtype, 42, first, n, 1.5, 0.5))
    buf = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    cuts = [0, 1, 2, 3, 1000, 1001, 65537, 100000, n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        gpu_fill(dist, dtype, 42, first + a, b - a, 1.5, 0.5, out=buf[a:b])
    got = to_np(buf)
    it = np.int64 if dtype == F64 else np.int32
    assert np.array_equal(got.view(it), whole.view(it))


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_edges(O, torch_cuda, dist, dtype):
    """n = 0 leaves the buffer alone; n = 1; the top of the index space;
    an output pointer that is not 16-byte aligned."""
    torch = torch_cuda
    from paper_1403_6870_amd import zig
    tdt = torch.float64 if dtype == F64 else torch.float32
    buf = torch.full((16,), 7.0, dtype=tdt, device="cuda")
    zig.zig_fill(dist, dtype, 1, 0, 0, 1.0, 1.0, buf.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert bool((buf == 7.0).all())
    p0, p1 = (1.0, 0.0) if dist == EXP else (0.0, 1.0)
    for first, n in [(0, 1), (5, 1), (2 ** 64 - 5, 5), (2 ** 64 - 1, 1), (2 ** 63 + 3, 1000)]:
        got = to_np(gpu_fill(dist, dtype, 3, first, n, p0, p1))
        want = oracle_fill(O, dist, dtype, 3, first, n, p0, p1)
        parity(got, want, ULP[dtype])
    big = torch.empty(5001, dtype=tdt, device="cuda")
    for off in (1, 2, 3):
        view = big[off:off + 4000]
        gpu_fill(dist, dtype, 8, 10, 4000, p0, p1, out=view)
        want = oracle_fill(O, dist, dtype, 8, 10, 4000, p0, p1)
        parity(to_np(view), want, ULP[dtype])


def _chunks(n, k, size, rng):
    starts = [0, n - size] + sorted(int(v) for v in rng.integers(0, n - size, size=k))
    return [(s, size) for s in starts]


@pytest.mark.parametrize("dtype", [F64, F32])
def test_c2_normal_2_28_sampled(O, torch_cuda, dtype):
    """N(0,1), 2^28 samples, seed 7, one launch (FP64: 2 GiB): sampled chunks
    (head, tail, 32 random) against the oracle; mean and variance of all
    outputs within 4.5 standard errors."""
    torch = torch_cuda
    n = 1 << 28
    out = gpu_fill(NORMAL, dtype, 7, 0, n, 0.0, 1.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for s, size in _chunks(n, 32, 1 << 14, rng):
        got = out[s:s + size].cpu().numpy()
        want = oracle_fill(O, NORMAL, dtype, 7, s, size, 0.0, 1.0)
        parity(got, want, ULP[dtype])
    x = out.double()
    m = float(x.mean())
    v = float(x.var())
    del x
    assert abs(m) < 4.5 / n ** 0.5
    assert abs(v - 1) < 4.5 * (2.0 / n) ** 0.5


def _full_parity(O, torch, dist, dtype, seed, n, p0, p1):
    out = gpu_fill(dist, dtype, seed, 0, n, p0, p1)
    torch.cuda.synchronize()
    chunk = 1 << 26
    total_nd, total_mu = 0, 0
    for s in range(0, n, chunk):
        got = out[s:s + chunk].cpu().numpy()
        want = oracle_fill(O, dist, dtype, seed, s, min(chunk, n - s), p0, p1)
        nd, mu = parity(got, want, ULP[dtype])
        total_nd += nd
        total_mu = max(total_mu, mu)
    del out
    torch.cuda.empty_cache()
    return total_nd, total_mu


@pytest.mark.slow
def test_c3_exp_2_30_full_parity(O, torch_cuda):
    """Exp(lambda = 2.5), 2^30 FP64 samples, seed 11: every output against
    the oracle (over 10^9 draws; no decision may differ)."""
    nd, mu = _full_parity(O, torch_cuda, EXP, F64, 11, 1 << 30, 2.5, 0.0)
    _report("c3 exp f64 full", nd, mu)
    assert nd == 0


@pytest.mark.slow
def test_c3_normal_2_30_full_parity(O, torch_cuda):
    """N(mu = -1, sigma = 3), 2^30 FP64 samples, seed 12, every output."""
    nd, mu = _full_parity(O, torch_cuda, NORMAL, F64, 12, 1 << 30, -1.0, 3.0)
    _report("c3 normal f64 full", nd, mu)
    assert nd == 0


@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_c3_fp32_2_30_sampled(O, torch_cuda, dist):
    """The FP32 variants of the 2^30 fills: sampled chunks within 2 ulp."""
    torch = torch_cuda
    n = 1 << 30
    seed = 11 if dist == EXP else 12
    p0, p1 = (2.5, 0.0) if dist == EXP else (-1.0, 3.0)
    out = gpu_fill(dist, F32, seed, 0, n, p0, p1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for s, size in _chunks(n, 32, 1 << 14, rng):
        got = out[s:s + size].cpu().numpy()
        want = oracle_fill(O, dist, F32, seed, s, size, p0, p1)
        parity(got, want, ULP[F32])
    del out
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_c2_normal_2_28_full_parity(O, torch_cuda):
    """N(0,1), 2^28 FP64 samples, seed 7, one launch: every output."""
    nd, mu = _full_parity(O, torch_cuda, NORMAL, F64, 7, 1 << 28, 0.0, 1.0)
    _report("c2 normal f64 full", nd, mu)
    assert nd == 0


@pytest.mark.slow
@pytest.mark.parametrize("dist", [EXP, NORMAL])
def test_c3_fp32_2_30_full_parity(O, torch_cuda, dist):
    """The FP32 variants of the 2^30 fills (Appendix D item 4's single
    precision), seeds 11 and 12: every output within 2 ulp."""
    seed = 11 if dist == EXP else 12
    p0, p1 = (2.5, 0.0) if dist == EXP else (-1.0, 3.0)
    nd, mu = _full_parity(O, torch_cuda, dist, F32, seed, 1 << 30, p0, p1)
    _report("c3 d%d f32 full" % dist, nd, mu)


def test_captured_fills_replay_concurrently(torch_cuda):
    """Fills captured into graphs hold no scratch: two graphs (large fills
    that would take tile counters outside a capture) replayed at the same
    time on two streams, several times with eager work between, give the
    eager outputs bit for bit."""
    from paper_1403_6870_amd import zig
    torch = torch_cuda
    n = (1 << 25) + 3
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    ref_a = to_np(gpu_fill(NORMAL, F64, 5, 9, n, -1.0, 3.0, out=a)).copy()
    ref_b = to_np(gpu_fill(EXP, F64, 6, 2, n, 2.5, 0.0, out=b)).copy()
    cap = torch.cuda.Stream()
    g1, g2 = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g1, stream=cap):
        zig.fill(a, NORMAL, 5, 9, -1.0, 3.0, stream=cap)
    with torch.cuda.graph(g2, stream=cap):
        zig.fill(b, EXP, 6, 2, 2.5, 0.0, stream=cap)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        a.zero_()
        b.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            g1.replay()
        with torch.cuda.stream(s2):
            g2.replay()
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy().view(np.int64), ref_a.view(np.int64))
        assert np.array_equal(b.cpu().numpy().view(np.int64), ref_b.view(np.int64))


def test_capture_allocates_nothing(O, torch_cuda):
    """Under graph capture a fill allocates and copies nothing: with no
    tables of its i_max on the device (32 layers, used by no other GPU
    test) it returns ZIG_ESTATE, and a batch is refused on the capturing
    stream, both without breaking the capture, whose other fill replays
    bit for bit.  Once zig_build_tables(32) has run, the same fill captures
    and replays as it runs eagerly."""
    from paper_1403_6870_amd import zig
    torch = torch_cuda
    n = 5003
    ok = torch.empty(n, dtype=torch.float64, device="cuda")
    small = torch.empty(n, dtype=torch.float64, device="cuda")
    ref_ok = to_np(gpu_fill(NORMAL, F64, 4, 7, n, 0.5, 2.0, out=ok)).copy()
    cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cap):
        with pytest.raises(zig.ZigError) as e:
            zig.fill(small, EXP, 4, 0, 1.0, 0.0, launch={"i_max": 32}, stream=cap)
        assert e.value.status == zig.ZIG_ESTATE and "zig_build_tables" in str(e.value)
        with pytest.raises(zig.ZigError) as e:
            zig.fill_batch([(small, EXP, 4, 0, 1.0, 0.0)], stream=cap)
        assert e.value.status == zig.ZIG_EINVAL and "captured" in str(e.value)
        zig.fill(ok, NORMAL, 4, 7, 0.5, 2.0, stream=cap)
    for _ in range(2):
        ok.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ok.cpu().numpy().view(np.int64), ref_ok.view(np.int64))

    zig.zig_build_tables(32)
    ref_small = to_np(gpu_fill(EXP, F64, 4, 0, n, 1.0, 0.0, out=small, launch={"i_max": 32})).copy()
    parity(ref_small, oracle_fill(O, EXP, F64, 4, 0, n, 1.0, 0.0, i_max=32), ULP[F64])
    g2 = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g2, stream=cap):
        zig.fill(small, EXP, 4, 0, 1.0, 0.0, launch={"i_max": 32}, stream=cap)
    for _ in range(2):
        small.zero_()
        torch.cuda.synchronize()
        g2.replay()
        torch.cuda.synchronize()
        assert np.array_equal(small.cpu().numpy().view(np.int64), ref_small.view(np.int64))


def test_per_thread_streams_from_many_threads(torch_cuda):
    """Large fills (counter-scheduled) on the per-thread stream handle from
    four host threads at once: each launch has its own counter pair, so
    every output equals its fill alone."""
    import ctypes
    import threading

    from paper_1403_6870_amd import zig
    torch = torch_cuda
    n = (1 << 24) + 5
    bufs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    refs = [to_np(gpu_fill(k % 2, F64, 70 + k, 0, n, 1.5, 0.5)).copy() for k in range(4)]
    errors = []
    launch = zig.Launch(0, 64, 1, 0)  # 64-block tiles: far above the static threshold

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    per_thread = ctypes.c_void_p(2)  # hipStreamPerThread

    def work(k):
        try:
            for _ in range(5):
                zig.zig_fill(k % 2, F64, 70 + k, 0, n, 1.5, 0.5, bufs[k].data_ptr(), 2, launch)
            # the thread's own stream is synchronised before the thread ends;
            # a device-wide synchronisation afterwards need not cover it
            rc = hip.hipStreamSynchronize(per_thread)
            assert rc == 0, rc
        except Exception as e:  # reported below
            errors.append(e)

    torch.cuda.synchronize()
    ts = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for k in range(4):
        got = bufs[k].cpu().numpy().view(np.int64)
        bad = np.flatnonzero(got != refs[k].view(np.int64))
        assert len(bad) == 0, (k, len(bad), bad[:8].tolist())


def test_counter_ring_reuse_across_streams(torch_cuda):
    """More counter-scheduled launches than the ring has slots, alternating
    between two streams and two buffers: the final outputs are exact."""
    from paper_1403_6870_amd import zig
    torch = torch_cuda
    n = (1 << 22) + 1
    ref = to_np(gpu_fill(NORMAL, F64, 3, 1, n, 0.0, 1.0)).copy()
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    launch = {"wg": 64, "spl": 1}
    torch.cuda.synchronize()
    for k in range(150):
        zig.fill(outs[k % 2], NORMAL, 3, 1, 0.0, 1.0, launch=launch, stream=streams[k % 2])
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy().view(np.int64), ref.view(np.int64))
