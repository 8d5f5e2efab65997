"""GPU tests of the batched fill: every request of a batch is bit-identical
to the same request filled alone (and, sampled, to the oracle), on the graph
and direct paths, for every batch shape, across repeated graph replays with
other device work in between."""
import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL, oracle_fill, parity, to_np

pytestmark = pytest.mark.gpu

BATCH_SHAPES = [(64, 4), (128, 4), (128, 8), (256, 2), (256, 4), (512, 2)]


def mixed_requests(rng, count, max_log2, fp32_share=0.5):
    """Sizes floor(2^(max_log2 U)), dist Bernoulli(1/2), exp lambda ~
    U[0.1, 10], normal mu ~ N(0,1), sigma ~ U[0.1, 5], seed = request id."""
    out = []
    for k in range(count):
        n = int(np.floor(2.0 ** (max_log2 * rng.random())))
        dist = int(rng.random() < 0.5)
        dtype = int(rng.random() < fp32_share)
        if dist == EXP:
            p0, p1 = float(rng.uniform(0.1, 10.0)), 0.0
        else:
            p0, p1 = float(rng.normal()), float(rng.uniform(0.1, 5.0))
        first = int(rng.integers(0, 1000)) if rng.random() < 0.3 else 0
        out.append((dist, dtype, k, first, n, p0, p1))
    return out


def _alloc(torch, reqs):
    return [torch.empty(max(n, 1), dtype=torch.float64 if dt == F64 else torch.float32, device="cuda")[:n]
            for (_, dt, _, _, n, _, _) in reqs]


def _single(torch, zig, reqs):
    outs = _alloc(torch, reqs)
    for (dist, dt, seed, first, n, p0, p1), o in zip(reqs, outs):
        if n:
            zig.fill(o, dist, seed, first, p0, p1)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def _batch(torch, zig, reqs, opts=None):
    outs = _alloc(torch, reqs)
    arr = (zig.Request * len(reqs))()
    for k, ((dist, dt, seed, first, n, p0, p1), o) in enumerate(zip(reqs, outs)):
        arr[k] = zig.Request(dist, dt, seed, first, n, p0, p1, o.data_ptr() if n else None)
    zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream, opts)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def _same(a, b):
    for x, y in zip(a, b):
        it = np.int64 if x.dtype == np.float64 else np.int32
        if not np.array_equal(x.view(it), y.view(it)):
            return False
    return True


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_fills(O, env, graph):
    torch, zig = env
    rng = np.random.default_rng(4)
    reqs = mixed_requests(rng, 600, 16)
    reqs += [(EXP, F64, 9001, 5, 0, 1.0, 0.0), (NORMAL, F32, 9002, 1, 1, 0.0, 1.0),
             (NORMAL, F64, 9003, 2 ** 64 - 40, 40, -2.0, 0.5), (EXP, F32, 9004, 3, 3 * 4096 + 7, 3.0, 0.0)]
    want = _single(torch, zig, reqs)
    opts = None if graph else {"flags": zig.BATCH_NO_GRAPH}
    got = _batch(torch, zig, reqs, opts)
    assert _same(got, want)
    # sampled against the oracle
    for k in list(range(0, len(reqs), 37)) + [len(reqs) - 2, len(reqs) - 1]:
        dist, dt, seed, first, n, p0, p1 = reqs[k]
        if n:
            parity(got[k], oracle_fill(O, dist, dt, seed, first, n, p0, p1), 4 if dt == F64 else 2)


@pytest.mark.parametrize("wg,spl", BATCH_SHAPES)
def test_large_batch_lean_layout(env, wg, spl):
    """A batch of about 5e7 outputs: many tiles per resident workgroup at
    every shape, so the kernel reads the slow-path tables from device
    memory (the small batches above run the layout that stages them in
    LDS); outputs bit-identical to single fills."""
    torch, zig = env
    rng = np.random.default_rng(100 + wg + spl)
    reqs = mixed_requests(rng, 200, 22)
    assert sum(r[4] for r in reqs) > 4 * 10 ** 7
    want = _single(torch, zig, reqs)
    got = _batch(torch, zig, reqs, {"wg": wg, "spl": spl})
    assert _same(got, want)


@pytest.mark.parametrize("wg,spl", BATCH_SHAPES)
def test_batch_shapes(env, wg, spl):
    torch, zig = env
    rng = np.random.default_rng(wg * 10 + spl)
    reqs = mixed_requests(rng, 200, 15)
    want = _single(torch, zig, reqs)
    got = _batch(torch, zig, reqs, {"wg": wg, "spl": spl})
    assert _same(got, want)


def test_graph_replays_with_eager_work_between(env):
    """The same graph (same slot ring, same size bucket) replayed many times,
    with unrelated device work and synchronisations in between; every replay
    is checked against the single-fill result."""
    torch, zig = env
    rng = np.random.default_rng(7)
    scratch = torch.zeros(1 << 20, device="cuda")
    for rep in range(10):
        reqs = mixed_requests(rng, 300, 14)
        want = _single(torch, zig, reqs)
        scratch.add_(1.0)
        torch.cuda.synchronize()
        got = _batch(torch, zig, reqs)
        assert _same(got, want), rep
        float(scratch.sum())


def test_batch_overlaps_stream_and_ring(env):
    """Back-to-back batches without synchronisation reuse the slot ring; all
    results stay correct."""
    torch, zig = env
    rng = np.random.default_rng(8)
    batches = [mixed_requests(rng, 150, 14) for _ in range(9)]
    wants = [_single(torch, zig, r) for r in batches]
    outs_all = []
    for reqs in batches:
        outs = _alloc(torch, reqs)
        arr = (zig.Request * len(reqs))()
        for k, ((dist, dt, seed, first, n, p0, p1), o) in enumerate(zip(reqs, outs)):
            arr[k] = zig.Request(dist, dt, seed, first, n, p0, p1, o.data_ptr() if n else None)
        zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream)
        outs_all.append(outs)
    torch.cuda.synchronize()
    for outs, want in zip(outs_all, wants):
        assert _same([o.cpu().numpy() for o in outs], want)


def test_batch_invalid_request_rejected(env):
    torch, zig = env
    o = torch.empty(10, dtype=torch.float64, device="cuda")
    arr = (zig.Request * 3)(zig.Request(0, 0, 1, 0, 10, 1.0, 0.0, o.data_ptr()),
                            zig.Request(1, 0, 1, 0, 10, 0.0, -1.0, o.data_ptr()),
                            zig.Request(0, 0, 1, 0, 10, 1.0, 0.0, o.data_ptr()))
    with pytest.raises(zig.ZigError) as e:
        zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == zig.ZIG_EINVAL and "request 1" in str(e.value)


def test_batch_unknown_flag_rejected(env):
    torch, zig = env
    o = torch.empty(10, dtype=torch.float64, device="cuda")
    arr = (zig.Request * 1)(zig.Request(0, 0, 1, 0, 10, 1.0, 0.0, o.data_ptr()))
    with pytest.raises(zig.ZigError) as e:
        zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream, {"flags": 4})
    assert e.value.status == zig.ZIG_EINVAL


def test_rejected_batch_leaves_slots_usable(env):
    """Descriptors are written into the slot as the requests are checked:
    a large batch rejected at request 20 launches nothing, and the batches
    after it (more than the four slots, on and off the graph path) match
    the single fills bit for bit."""
    torch, zig = env
    reqs = mixed_requests(np.random.default_rng(9), 40, 14)
    outs = _alloc(torch, reqs)
    arr = (zig.Request * (len(reqs) + 1))()
    for k, ((dist, dt, seed, first, n, p0, p1), o) in enumerate(zip(reqs, outs)):
        arr[k if k < 20 else k + 1] = zig.Request(dist, dt, seed, first, n, p0, p1, o.data_ptr() if n else None)
    arr[20] = zig.Request(1, 0, 99, 0, 10, 0.0, -1.0, outs[0].data_ptr())  # sigma < 0
    with pytest.raises(zig.ZigError) as e:
        zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == zig.ZIG_EINVAL and "request 20" in str(e.value)
    want = _single(torch, zig, reqs)
    for k in range(6):
        opts = {"flags": zig.BATCH_NO_GRAPH} if k % 2 else None
        assert _same(_batch(torch, zig, reqs, opts), want), k


def c4_requests(count=4096):
    """The 4096-request mixed batch: per request, in this order from
    numpy.random.default_rng(4), size floor(2^(20 U)), dist Bernoulli(1/2),
    then exp lambda ~ U[0.1, 10] or normal mu ~ N(0, 1), sigma ~ U[0.1, 5];
    FP64, seed = request id, first index 0."""
    rng = np.random.default_rng(4)
    out = []
    for k in range(count):
        n = int(np.floor(2.0 ** (20.0 * rng.random())))
        dist = int(rng.random() < 0.5)
        if dist == EXP:
            p0, p1 = float(rng.uniform(0.1, 10.0)), 0.0
        else:
            p0, p1 = float(rng.normal()), float(rng.uniform(0.1, 5.0))
        out.append((dist, F64, k, 0, n, p0, p1))
    return out


@pytest.mark.slow
def test_c4_batch_full_parity(O, env):
    """The 4096-request batch (3.0e8 FP64 outputs) in one graph launch of
    the tuned shape: every output of every request against the oracle, no
    decision may differ."""
    torch, zig = env
    reqs = c4_requests()
    offs, tot = [], 0
    for r in reqs:
        offs.append(tot)
        tot += r[4] + (r[4] & 1)
    arena = torch.empty(tot, dtype=torch.float64, device="cuda")
    arr = (zig.Request * len(reqs))()
    for k, (dist, dt, seed, first, n, p0, p1) in enumerate(reqs):
        arr[k] = zig.Request(dist, dt, seed, first, n, p0, p1, arena.data_ptr() + 8 * offs[k] if n else None)
    zig.zig_fill_batch(arr, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    host = arena.cpu().numpy()
    del arena
    torch.cuda.empty_cache()
    total_nd, total_mu, samples = 0, 0, 0
    for k, (dist, dt, seed, first, n, p0, p1) in enumerate(reqs):
        if n == 0:
            continue
        nd, mu = parity(host[offs[k]:offs[k] + n], oracle_fill(O, dist, dt, seed, first, n, p0, p1), 4)
        total_nd += nd
        total_mu = max(total_mu, mu)
        samples += n
    print("c4 batch full: %d outputs, %d not bit-identical, max %d ulp" % (samples, total_nd, total_mu), flush=True)
    assert samples == sum(r[4] for r in reqs) and total_nd == 0
