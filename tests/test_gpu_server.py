"""GPU tests of the serving loop on the device backend: every served
request equals zig_fill of (seed_base + client, first_index) bit for bit,
whatever it was batched with; first indices follow each client's submission
order; the device counters match that rule; checkpoint/restore continues a
client's stream; the open-loop replays (batched and naive) return the same
samples as fills of the reported indices."""
import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL, oracle_fill, parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


def served_view(torch, arena, c):
    off = c.out - arena.data_ptr()
    es = 8 if c.dtype == F64 else 4
    raw = arena[off:off + c.n * es]
    return raw.view(torch.float64 if c.dtype == F64 else torch.float32)


def alone(torch, zig, c, p0, p1):
    t = torch.empty(c.n, dtype=torch.float64 if c.dtype == F64 else torch.float32, device="cuda")
    zig.fill(t, c.dist, c.seed, c.first_index, p0, p1)
    return t


def random_specs(rng, count, clients, max_log2):
    out = []
    for _ in range(count):
        c = int(rng.integers(0, clients))
        dist = int(rng.integers(0, 2))
        dt = int(rng.integers(0, 2))
        n = int(np.floor(2.0 ** (max_log2 * rng.random())))
        if dist == EXP:
            p0, p1 = float(rng.uniform(0.1, 10.0)), 0.0
        else:
            p0, p1 = float(rng.normal()), float(rng.uniform(0.1, 5.0))
        out.append((c, dist, dt, n, p0, p1))
    return out


@pytest.mark.parametrize("streams,max_batch", [(4, 1024), (2, 5), (1, 1)])
def test_served_equals_alone(env, streams, max_batch):
    torch, zig = env
    cap = 1 << 28
    arena = torch.empty(cap, dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(100 + streams)
    specs = random_specs(rng, 400, 8, 16)
    with zig.Server(cap, streams=streams, max_batch=max_batch, clients=8, seed_base=1000,
                    arena_ptr=arena.data_ptr()) as s:
        tickets = [s.submit(c, d, dt, n, p0, p1) for (c, d, dt, n, p0, p1) in specs]
        nxt = [0] * 8
        for (c, d, dt, n, p0, p1), t in zip(specs, tickets):
            comp = s.wait(t)
            assert comp.status == 0 and comp.seed == 1000 + c
            assert comp.first_index == nxt[c]
            nxt[c] += n
            if n:
                got = served_view(torch, arena, comp)
                assert torch.equal(got, alone(torch, zig, comp, p0, p1)), (c, d, dt, n)
            s.release(t)
        assert list(s.counters()) == nxt
        st = s.stats()
        assert st["bytes_in_use"] == 0 and st["failed_requests"] == 0


def test_served_matches_oracle_sampled(O, env):
    torch, zig = env
    cap = 1 << 26
    arena = torch.empty(cap, dtype=torch.uint8, device="cuda")
    specs = [(0, EXP, F64, 1000, 2.5, 0.0), (1, NORMAL, F32, 777, -1.0, 3.0), (0, NORMAL, F64, 4097, 0.5, 0.25),
             (1, EXP, F32, 33, 0.3, 0.0)]
    with zig.Server(cap, clients=2, seed_base=77, arena_ptr=arena.data_ptr()) as s:
        tickets = [s.submit(*sp) for sp in specs]
        for (c, d, dt, n, p0, p1), t in zip(specs, tickets):
            comp = s.wait(t)
            got = served_view(torch, arena, comp).cpu().numpy()
            parity(got, oracle_fill(O, d, dt, 77 + c, comp.first_index, n, p0, p1), 4 if dt == F64 else 2)
            s.release(t)


def test_device_counters_checkpoint_restore(env):
    torch, zig = env
    cap = 1 << 24
    with zig.Server(cap, clients=3, seed_base=5) as s:
        for c, n in [(0, 100), (1, 7), (0, 3), (2, 4096), (1, 1)]:
            t = s.submit(c, EXP, F64, n, 1.0)
            s.wait(t)
            s.release(t)
        snap = s.counters()
    assert list(snap) == [103, 8, 4096]
    arena = torch.empty(cap, dtype=torch.uint8, device="cuda")
    with zig.Server(cap, clients=3, seed_base=5, arena_ptr=arena.data_ptr()) as s2:
        s2.set_counters(snap)
        t = s2.submit(2, NORMAL, F32, 1000, 0.0, 1.0)
        comp = s2.wait(t)
        assert comp.first_index == 4096
        assert torch.equal(served_view(torch, arena, comp), alone(torch, zig, comp, 0.0, 1.0))
        s2.release(t)
        assert list(s2.counters()) == [103, 8, 5096]


def test_index_overflow_rejected_on_device(env):
    torch, zig = env
    top = 2 ** 64 - 1
    arena = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with zig.Server(1 << 20, clients=1, arena_ptr=arena.data_ptr()) as s:
        s.set_counters([top - 50])
        t = s.submit(0, EXP, F64, 50, 1.0)
        comp = s.wait(t)
        assert comp.first_index == top - 50
        assert torch.equal(served_view(torch, arena, comp), alone(torch, zig, comp, 1.0, 0.0))
        s.release(t)
        st, _ = s.poll(s.submit(0, EXP, F64, 1, 1.0))
        assert st == zig.ZIG_EINVAL
        assert list(s.counters()) == [top]


@pytest.mark.parametrize("naive", [False, True])
def test_replay_outputs(env, naive):
    torch, zig = env
    rng = np.random.default_rng(55)
    m = 600
    tr = np.zeros(m, dtype=zig.TRACE_DTYPE)
    tr["client"] = rng.integers(0, 16, m)
    tr["dist"] = rng.integers(0, 2, m)
    tr["dtype"] = rng.integers(0, 2, m)
    tr["n"] = np.floor(2.0 ** (4 + 14 * rng.random(m))).astype(np.uint64)
    tr["p0"] = np.where(tr["dist"] == EXP, rng.uniform(0.1, 10.0, m), rng.normal(size=m))
    tr["p1"] = np.where(tr["dist"] == EXP, 0.0, rng.uniform(0.1, 5.0, m))
    tr["t_arrival_ns"] = np.cumsum(rng.exponential(50000.0, m)).astype(np.uint64)
    sel = np.flatnonzero(rng.random(m) < 0.2)
    copies = {}
    for i in sel:
        t = torch.empty(int(tr["n"][i]), dtype=torch.float64 if tr["dtype"][i] == F64 else torch.float32,
                        device="cuda")
        copies[i] = t
        tr["copy_to"][i] = t.data_ptr()
    with zig.Server(1 << 30, clients=16, seed_base=1000) as s:
        out = s.replay(tr, naive=naive)
        assert s.stats()["bytes_in_use"] == 0
    assert np.all(out["status"] == 0)
    assert np.all(out["t_done_ns"] >= out["t_arrival_ns"])
    nxt = np.zeros(16, dtype=np.uint64)
    for i in range(m):
        c = tr["client"][i]
        assert out["first_index"][i] == nxt[c]
        nxt[c] += tr["n"][i]
    torch.cuda.synchronize()
    for i, t in copies.items():
        want = torch.empty_like(t)
        zig.fill(want, int(tr["dist"][i]), 1000 + int(tr["client"][i]), int(out["first_index"][i]),
                 float(tr["p0"][i]), float(tr["p1"][i]))
        assert torch.equal(t, want), i
