"""Scheduler tests of the serving loop on the host fake backend (no device
calls): index assignment in admission order, admission against the output
cap, status codes for invalid requests, injected failures that use no
index, client disconnect, counter checkpoint/restore, open-loop replay.

The fake writes first_index + k as the k-th output, so every test can read
back which indices a request was given."""
import ctypes
import threading
import time

import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL


@pytest.fixture(scope="module")
def zig():
    from paper_1403_6870_amd import zig as z
    return z


def fake(zig, **kw):
    kw.setdefault("cap_bytes", 1 << 22)
    return zig.Server(backend=zig.BACKEND_HOST_FAKE, **kw)


def values(c):
    n = c.n
    if n == 0:
        return np.zeros(0)
    t = ctypes.c_double if c.dtype == F64 else ctypes.c_float
    return np.ctypeslib.as_array((t * n).from_address(c.out)).astype(np.float64)


def expect_indices(c):
    return np.arange(c.first_index, c.first_index + c.n, dtype=np.float64)


def test_indices_follow_submission_order_per_client(zig):
    rng = np.random.default_rng(1)
    with fake(zig, clients=5, max_batch=7, streams=2, fake_latency_us=200) as s:
        reqs = []
        for _ in range(200):
            c = int(rng.integers(0, 5))
            n = int(rng.integers(1, 300))
            dt = int(rng.integers(0, 2))
            reqs.append((c, n, dt, s.submit(c, EXP, dt, n, 1.5)))
        nxt = [0] * 5
        for c, n, dt, t in reqs:
            comp = s.wait(t)
            assert comp.status == 0 and comp.client == c and comp.n == n
            assert comp.first_index == nxt[c], (c, comp.first_index, nxt[c])
            assert comp.batch_size <= 7
            assert comp.t_arrival_ns <= comp.t_submit_ns <= comp.t_admit_ns <= comp.t_launch_ns <= comp.t_done_ns
            np.testing.assert_array_equal(values(comp), expect_indices(comp))
            nxt[c] += n
            s.release(t)
        assert list(s.counters()) == nxt
        st = s.stats()
        assert st["requests"] == 200 and st["bytes_in_use"] == 0 and st["queued"] == 0
        assert st["batches"] >= 200 / 7


def test_seed_per_client(zig):
    with fake(zig, clients=3, seed_base=1000) as s:
        t = s.submit(2, NORMAL, F64, 4, 0.0, 1.0)
        assert s.wait(t).seed == 1002


def test_admission_blocks_at_tiny_cap(zig):
    cap = 4096
    with fake(zig, cap_bytes=cap, fake_latency_us=2000, streams=2) as s:
        tickets = [s.submit(0, EXP, F64, 128, 1.0) for _ in range(24)]  # 1 KiB each
        # non-blocking submission is refused while admitted + queued exceed the cap
        with pytest.raises(zig.ZigError) as e:
            s.submit(0, EXP, F64, 128, 1.0, nonblock=True)
        assert e.value.status == zig.ZIG_EBUSY
        time.sleep(0.01)
        st = s.stats()
        assert st["bytes_in_use"] <= cap and st["queued"] > 0
        nxt = 0
        for t in tickets:  # waiting + releasing in order drains the queue
            c = s.wait(t)
            assert c.first_index == nxt
            nxt += 128
            assert s.stats()["bytes_in_use"] <= cap
            s.release(t)
        st = s.stats()
        assert st["max_bytes_in_use"] <= cap and st["bytes_in_use"] == 0
        s.submit(0, EXP, F64, 128, 1.0, nonblock=True)


def test_unreleased_outputs_hold_admission(zig):
    with fake(zig, cap_bytes=2048) as s:
        a = s.submit(0, EXP, F64, 256, 1.0)  # the whole cap
        ca = s.wait(a)
        b = s.submit(0, EXP, F64, 1, 1.0)
        with pytest.raises(zig.ZigError) as e:
            s.wait(b, timeout_us=20000)
        assert e.value.status == zig.ZIG_EBUSY  # timed out: not admitted
        s.release(a)
        cb = s.wait(b, timeout_us=2_000_000)
        assert cb.first_index == ca.first_index + 256


@pytest.mark.parametrize("dist,p0,p1", [(EXP, 0.0, 0.0), (EXP, -1.0, 0.0), (EXP, float("nan"), 0.0),
                                        (EXP, float("inf"), 0.0), (NORMAL, 0.0, 0.0), (NORMAL, 0.0, -2.0),
                                        (NORMAL, float("nan"), 1.0), (NORMAL, 0.0, float("nan")),
                                        (NORMAL, float("inf"), 1.0)])
def test_invalid_parameters(zig, dist, p0, p1):
    with fake(zig) as s:
        with pytest.raises(zig.ZigError) as e:
            s.submit(0, dist, F64, 10, p0, p1)
        assert e.value.status == zig.ZIG_EINVAL
        assert s.stats()["queued"] == 0


def test_invalid_requests(zig):
    with fake(zig, cap_bytes=1024, clients=4) as s:
        for args in [(4, EXP, F64, 1), (0, 2, F64, 1), (0, EXP, 2, 1), (0, EXP, F64, 129), (0, EXP, F32, 257)]:
            with pytest.raises(zig.ZigError) as e:
                s.submit(*args, 1.0)
            assert e.value.status == zig.ZIG_EINVAL, args
        s.submit(0, EXP, F32, 256, 1.0)  # exactly the cap is fine
        with pytest.raises(zig.ZigError) as e:
            s.release(12345)
        assert e.value.status == zig.ZIG_ESTATE
        with pytest.raises(zig.ZigError) as e:
            s.wait(12345)
        assert e.value.status == zig.ZIG_ESTATE


def test_index_overflow_rejected_without_advancing(zig):
    top = 2 ** 64 - 1
    with fake(zig, clients=2) as s:
        s.set_counters([top - 100, 7])
        ok = s.submit(0, EXP, F64, 100, 1.0)  # last index 2^64 - 2
        c = s.wait(ok)
        assert c.first_index == top - 100
        assert values(c)[-1] == float(top - 1)
        bad = s.submit(0, EXP, F64, 1, 1.0)
        st, cb = s.poll(bad)
        assert st == zig.ZIG_EINVAL and cb.status == zig.ZIG_EINVAL and cb.out is None
        other = s.wait(s.submit(1, EXP, F64, 3, 1.0))
        assert other.first_index == 7
        assert list(s.counters()) == [top, 10]


def test_injected_failures_use_no_index(zig):
    with fake(zig, fake_fail_every=3, max_batch=4) as s:
        tickets = [s.submit(0, EXP, F64, 10, 1.0) for _ in range(9)]
        got = []
        for k, t in enumerate(tickets):
            st, c = s.poll(t)
            if (k + 1) % 3 == 0:
                assert st == zig.ZIG_EHIP and c.out is None
            else:
                assert st == zig.ZIG_OK
                np.testing.assert_array_equal(values(c), expect_indices(c))
                got.append(c.first_index)
            s.release(t)
        assert got == [0, 10, 20, 30, 40, 50]
        assert s.counters()[0] == 60
        assert s.stats()["failed_requests"] == 3


def test_zero_length_request(zig):
    with fake(zig) as s:
        t = s.submit(0, EXP, F64, 0, 1.0)
        c = s.wait(t)
        assert c.status == 0 and c.n == 0
        s.release(t)
        assert s.counters()[0] == 0


def test_release_before_completion_refused(zig):
    with fake(zig, fake_latency_us=50000) as s:
        t = s.submit(0, EXP, F64, 10, 1.0)
        with pytest.raises(zig.ZigError) as e:
            s.release(t)
        assert e.value.status == zig.ZIG_ESTATE
        s.wait(t)
        s.release(t)


def test_client_disconnect_reclaims_buffers(zig):
    with fake(zig, cap_bytes=8192, fake_latency_us=5000, streams=1, clients=3) as s:
        keep = [s.submit(0, EXP, F64, 64, 1.0) for _ in range(3)]
        gone = [s.submit(1, EXP, F64, 128, 1.0) for _ in range(10)]  # more than the cap: some queue
        s.wait(gone[0])  # a completed one, not released
        n = s.drop_client(1)
        assert n == 10
        for t in keep:
            s.wait(t)
            s.release(t)
        deadline = time.time() + 5
        while s.stats()["bytes_in_use"] and time.time() < deadline:
            time.sleep(0.005)
        st = s.stats()
        assert st["bytes_in_use"] == 0 and st["queued"] == 0 and st["inflight_batches"] == 0
        for t in gone:
            with pytest.raises(zig.ZigError):
                s.wait(t, timeout_us=0)
        # the client may come back; its counter kept what its launched requests used
        c = s.wait(s.submit(1, EXP, F64, 1, 1.0))
        assert c.first_index % 128 == 0 and c.first_index >= 128


def test_counter_checkpoint_and_restore(zig):
    with fake(zig, clients=4) as s:
        for c in range(4):
            for n in (5, 17):
                s.wait(s.submit(c, EXP, F64, n * (c + 1), 1.0))
        snap = s.counters()
    assert list(snap) == [22 * (c + 1) for c in range(4)]
    with fake(zig, clients=4) as s2:
        s2.set_counters(snap)
        c = s2.wait(s2.submit(3, NORMAL, F32, 9, 0.0, 1.0))
        assert c.first_index == snap[3]
        np.testing.assert_array_equal(values(c), expect_indices(c))
        # restore needs an idle server
        slow = fake(zig, clients=1, fake_latency_us=100000)
        try:
            t = slow.submit(0, EXP, F64, 1, 1.0)
            with pytest.raises(zig.ZigError) as e:
                slow.set_counters([5])
            assert e.value.status == zig.ZIG_ESTATE
            slow.wait(t)
        finally:
            slow.close()


def test_concurrent_submitters(zig):
    """Several host threads submitting for their own clients: each client's
    indices are contiguous in its own submission order."""
    with fake(zig, clients=8, max_batch=16, streams=3) as s:
        res = {}

        def run(c):
            rng = np.random.default_rng(c)
            mine = []
            for _ in range(100):
                n = int(rng.integers(1, 64))
                mine.append((n, s.submit(c, EXP, F32, n, 2.0)))
            out = []
            for n, t in mine:
                comp = s.wait(t)
                np.testing.assert_array_equal(values(comp), expect_indices(comp))
                out.append((comp.first_index, n))
                s.release(t)
            res[c] = out

        th = [threading.Thread(target=run, args=(c,)) for c in range(8)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for c in range(8):
            nxt = 0
            for first, n in res[c]:
                assert first == nxt
                nxt += n
            assert s.counters()[c] == nxt


def test_replay_open_loop(zig):
    rng = np.random.default_rng(5)
    m = 300
    tr = np.zeros(m, dtype=zig.TRACE_DTYPE)
    tr["client"] = rng.integers(0, 4, m)
    tr["dist"] = rng.integers(0, 2, m)
    tr["dtype"] = rng.integers(0, 2, m)
    tr["n"] = rng.integers(1, 200, m)
    tr["p0"] = 1.0
    tr["p1"] = 1.0
    tr["t_arrival_ns"] = np.cumsum(rng.exponential(20000.0, m)).astype(np.uint64)
    keep = rng.random(m) < 0.1
    bufs = {}
    for i in np.flatnonzero(keep):
        b = np.zeros(int(tr["n"][i]), dtype=np.float64 if tr["dtype"][i] == F64 else np.float32)
        bufs[i] = b
        tr["copy_to"][i] = b.ctypes.data
    with fake(zig, clients=4, fake_latency_us=100) as s:
        out = s.replay(tr)
        assert s.stats()["bytes_in_use"] == 0
    assert np.all(out["status"] == 0)
    lat = (out["t_done_ns"] - out["t_arrival_ns"]).astype(np.int64)
    assert np.all(lat > 0)
    t0 = out["t_arrival_ns"][0] - tr["t_arrival_ns"][0]
    np.testing.assert_array_equal(out["t_arrival_ns"] - t0, tr["t_arrival_ns"])
    nxt = np.zeros(4, dtype=np.uint64)
    for i in range(m):
        c = tr["client"][i]
        assert out["first_index"][i] == nxt[c]
        nxt[c] += tr["n"][i]
    for i, b in bufs.items():
        f = int(out["first_index"][i])
        np.testing.assert_array_equal(b.astype(np.float64), np.arange(f, f + len(b), dtype=np.float64))
    with fake(zig) as s:
        with pytest.raises(zig.ZigError) as e:
            s.replay(tr[:3], naive=True)
        assert e.value.status == zig.ZIG_EINVAL
        bad = tr[:3].copy()
        bad["t_arrival_ns"] = [5, 3, 9]
        with pytest.raises(zig.ZigError):
            s.replay(bad)


def test_destroy_cancels_queue(zig):
    s = fake(zig, cap_bytes=1024, fake_latency_us=20000)
    for _ in range(20):
        s.submit(0, EXP, F64, 128, 1.0)
    t0 = time.time()
    s.close()
    assert time.time() - t0 < 5
    with pytest.raises(zig.ZigError):
        s.submit(0, EXP, F64, 1, 1.0)


def test_bad_configs(zig):
    for kw in [dict(cap_bytes=0), dict(streams=9), dict(max_batch=5000), dict(clients=(1 << 20) + 1),
               dict(backend=7)]:
        kw.setdefault("cap_bytes", 4096)
        with pytest.raises(zig.ZigError) as e:
            zig.Server(**{"backend": zig.BACKEND_HOST_FAKE, **kw})
        assert e.value.status == zig.ZIG_EINVAL, kw
