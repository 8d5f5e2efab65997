"""Benchmark of the gfx950 modified-ziggurat sampler.

One step = the plain fill at its largest single-GPU configuration, FP64:
2^30 Exp(lambda = 2.5) samples (seed 11) plus 2^30 N(mu = -1, sigma = 3)
samples (seed 12), each written once to a resident device buffer.  The
JSON line reports whole-job Gsamples/s, the HBM-write roofline of the fill
kernel (algorithmic bytes per launch over its average event-timed
duration), the CPU oracle timed on a bounded sample, and side numbers for
the other configurations (2^28 normal FP64; the FP32 variants; the batched
path against per-request launches).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# HBM bytes per launch of the normal FP64 fill kernel (2^30 outputs) from
# rocprofv3 FETCH_SIZE / WRITE_SIZE, each scaled by the ratio of the known
# bytes of a 1 GiB device copy to what the same counter read for it; the
# commands and raw readings are in profiles/fill_kernel_counters.txt.
# Reset to None whenever the fill kernel changes until it is re-measured.
TRAFFIC = 8595702911
N_C3 = 1 << 30
N_C2 = 1 << 28


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed_fills(torch, zig, calls, steps, warmup):
    """Runs `calls` (a list of (fn, bytes)) `steps` times after `warmup`
    passes; returns (wall seconds, per-launch event durations in ms, bytes
    per launch)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        for fn, _b in calls:
            fn()
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in calls]
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        for k, (fn, _b) in enumerate(calls):
            evs[s][k][0].record(stream)
            fn()
            evs[s][k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    durs = [[a.elapsed_time(b) for a, b in row] for row in evs]
    return wall, durs


def c4_requests(count=4096):
    """4096 requests: size floor(2^(20 U)), dist Bernoulli(1/2), exp lambda ~
    U[0.1, 10], normal mu ~ N(0, 1), sigma ~ U[0.1, 5], FP64, seed = request
    id, first index 0; drawn in that order per request from
    numpy.random.default_rng(4)."""
    rng = np.random.default_rng(4)
    reqs = []
    for k in range(count):
        n = int(np.floor(2.0 ** (20.0 * rng.random())))
        dist = int(rng.random() < 0.5)
        if dist == 0:
            p0, p1 = float(rng.uniform(0.1, 10.0)), 0.0
        else:
            p0, p1 = float(rng.normal()), float(rng.uniform(0.1, 5.0))
        reqs.append((dist, 0, k, 0, n, p0, p1))
    return reqs


def batch_bench(torch, zig, reps=20):
    """The 4096-request mixed batch: one batched launch (graph replay)
    against the same requests as per-request launches."""
    reqs = c4_requests()
    offs, tot = [], 0
    for r in reqs:
        offs.append(tot)
        tot += r[4] + (r[4] & 1)  # keep every output 16-byte aligned
    samples = sum(r[4] for r in reqs)
    arena_b = torch.empty(tot, dtype=torch.float64, device="cuda")
    arena_e = torch.empty(tot, dtype=torch.float64, device="cuda")

    def make(arena):
        arr = (zig.Request * len(reqs))()
        base = arena.data_ptr()
        for k, (dist, dt, seed, first, n, p0, p1) in enumerate(reqs):
            arr[k] = zig.Request(dist, dt, seed, first, n, p0, p1, base + 8 * offs[k])
        return arr

    rb, re_ = make(arena_b), make(arena_e)
    st = torch.cuda.current_stream()
    sp = st.cuda_stream
    for _ in range(3):
        zig.zig_fill_batch(rb, sp)
        zig.zig_fill_each(re_, sp)
    torch.cuda.synchronize()
    lat, host = [], []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(st)
        zig.zig_fill_batch(rb, sp)
        b.record(st)
        host.append((time.perf_counter() - t0) * 1e3)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    # per-request launches on one stream: completion time of every request
    # (events after each chunk of 64 requests), all submitted at time 0
    per_lat, makespans = [], []
    for _ in range(5):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(reqs) // 64 + 1)]
        evs[0].record(st)
        for c in range(0, len(reqs), 64):
            chunk = (zig.Request * min(64, len(reqs) - c))(*re_[c:c + 64])
            zig.zig_fill_each(chunk, sp)
            evs[c // 64 + 1].record(st)
        torch.cuda.synchronize()
        ends = [evs[0].elapsed_time(e) for e in evs[1:]]
        per_lat.append(np.repeat(ends, 64)[:len(reqs)])
        makespans.append(ends[-1])
    per_lat = np.concatenate(per_lat)
    # per-request launches spread round-robin over 4 streams
    streams = [torch.cuda.Stream() for _ in range(4)]
    torch.cuda.synchronize()
    ms4 = []
    for _ in range(5):
        a = torch.cuda.Event(enable_timing=True)
        a.record(st)
        for s_ in streams:
            s_.wait_event(a)
        for k in range(4):
            sub = (zig.Request * len(range(k, len(reqs), 4)))(*[re_[i] for i in range(k, len(reqs), 4)])
            zig.zig_fill_each(sub, streams[k].cuda_stream)
        ends = []
        for s_ in streams:
            e = torch.cuda.Event(enable_timing=True)
            e.record(s_)
            ends.append(e)
        torch.cuda.synchronize()
        ms4.append(max(a.elapsed_time(e) for e in ends))
    identical = bool(torch.equal(arena_b.view(torch.int64), arena_e.view(torch.int64)))
    del arena_b, arena_e
    torch.cuda.empty_cache()
    lat = np.array(lat)
    return {
        "workload": "4096 requests, sizes floor(2^(20U)), 50/50 Exp(U[0.1,10]) / N(N(0,1), U[0.1,5]), FP64, "
                    "seed = request id (numpy default_rng(4))",
        "samples": samples, "bytes": samples * 8,
        "batch_graph": {"p50_ms": round(float(np.percentile(lat, 50)), 4),
                        "p99_ms": round(float(np.percentile(lat, 99)), 4),
                        "Gsamples/s": round(samples / (float(np.median(lat)) * 1e-3) / 1e9, 2),
                        "host_submit_ms": round(float(np.median(host)), 4),
                        "latency_note": "every request of a batch completes with the batch"},
        "per_request_1_stream": {"makespan_ms": round(float(np.median(makespans)), 3),
                                 "p50_ms": round(float(np.percentile(per_lat, 50)), 3),
                                 "p99_ms": round(float(np.percentile(per_lat, 99)), 3)},
        "per_request_4_streams": {"makespan_ms": round(float(np.median(ms4)), 3)},
        "speedup_vs_per_request": round(float(np.median(makespans)) / float(np.median(lat)), 2),
        "outputs_identical": identical,
    }


def c5_trace(zig, seconds, rate=20000.0, clients=64, seed=5):
    """Open-loop serving trace: Poisson arrivals at `rate`/s for `seconds`,
    n = floor(2^(4 + 20U)), dist Bernoulli(1/2), exp lambda ~ U[0.1, 10],
    normal mu ~ N(0, 1), sigma ~ U[0.1, 5], dtype FP32/FP64 50/50, client
    uniform over 64; drawn as whole arrays in that order from
    numpy.random.default_rng(5)."""
    rng = np.random.default_rng(seed)
    m = int(round(seconds * rate))
    gaps = rng.exponential(1.0 / rate, m)
    u = rng.random(m)
    dist = (rng.random(m) < 0.5).astype(np.uint32)
    lam = rng.uniform(0.1, 10.0, m)
    mu = rng.normal(size=m)
    sigma = rng.uniform(0.1, 5.0, m)
    dtype = (rng.random(m) < 0.5).astype(np.uint32)
    client = rng.integers(0, clients, m).astype(np.uint32)
    tr = np.zeros(m, dtype=zig.TRACE_DTYPE)
    tr["client"] = client
    tr["dist"] = dist
    tr["dtype"] = dtype
    tr["n"] = np.floor(2.0 ** (4.0 + 20.0 * u)).astype(np.uint64)
    tr["p0"] = np.where(dist == 0, lam, mu)
    tr["p1"] = np.where(dist == 0, 0.0, sigma)
    tr["t_arrival_ns"] = np.round(np.cumsum(gaps) * 1e9).astype(np.uint64)
    return tr


def serve_run(torch, zig, tr, naive, check_share=0.01):
    """Replays `tr` through a fresh server (16 GiB cap, 64 clients, seed of
    client c = 1000 + c); a seeded 1% of the requests are copied out and
    re-generated alone with zig_fill at the reported first index."""
    m = len(tr)
    tr = tr.copy()
    sel = np.flatnonzero(np.random.default_rng(55).random(m) < check_share)
    es = np.where(tr["dtype"][sel] == 0, 8, 4).astype(np.uint64)
    nbytes = tr["n"][sel] * es
    offs = np.concatenate([[0], np.cumsum((nbytes + 255) // 256 * 256)])
    copy_buf = torch.empty(int(offs[-1]) + 256, dtype=torch.uint8, device="cuda")
    tr["copy_to"][sel] = copy_buf.data_ptr() + offs[:-1]
    with zig.Server(16 << 30, clients=64, seed_base=1000, streams=4) as srv:
        out = srv.replay(tr, naive=naive)
        stats = srv.stats()
    torch.cuda.synchronize()
    ok = bool(np.all(out["status"] == 0))
    identical = ok
    for k, i in enumerate(sel):
        n = int(tr["n"][i])
        dt = torch.float64 if tr["dtype"][i] == 0 else torch.float32
        got = copy_buf[int(offs[k]):int(offs[k]) + int(nbytes[k])].view(dt)
        want = torch.empty(n, dtype=dt, device="cuda")
        zig.fill(want, int(tr["dist"][i]), 1000 + int(tr["client"][i]), int(out["first_index"][i]),
                 float(tr["p0"][i]), float(tr["p1"][i]))
        if not torch.equal(got, want):
            identical = False
            break
    del copy_buf
    torch.cuda.empty_cache()
    lat = (out["t_done_ns"].astype(np.int64) - out["t_arrival_ns"].astype(np.int64)) / 1e6
    span = (int(out["t_done_ns"].max()) - int(out["t_arrival_ns"].min())) / 1e9
    samples = float(tr["n"].sum())
    res = {"requests": m, "all_ok": ok,
           "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
           "max_ms": round(float(lat.max()), 4), "Gsamples/s": round(samples / span / 1e9, 3),
           "span_s": round(span, 3), "checked": int(len(sel)), "outputs_identical": identical}
    if not naive:
        res["batches"] = int(stats["batches"])
        res["mean_batch"] = round(m / max(1, stats["batches"]), 2)
        res["max_bytes_in_use"] = int(stats["max_bytes_in_use"])
    return res


def serve_bench(torch, zig, seconds):
    out = {"workload": "open-loop Poisson arrivals, n = floor(2^(4+20U)), 50/50 Exp(U[0.1,10]) / "
                       "N(N(0,1), U[0.1,5]), FP32/FP64 50/50, 64 clients (seed 1000 + id), 16 GiB admission "
                       "cap, 4 fill streams (numpy default_rng(5))",
           "latency": "host time the completion is observed minus the scheduled arrival"}
    for name, rate, secs in [("rate_20k", 20000.0, seconds), ("rate_200k", 200000.0, min(2.0, seconds))]:
        tr = c5_trace(zig, secs, rate)
        offered = float(tr["n"].sum()) / secs / 1e9
        log("serve %s: %d requests over %.1f s (offered %.1f Gsamples/s)" % (name, len(tr), secs, offered))
        run = {"offered_Gsamples/s": round(offered, 3), "seconds": secs}
        run["batched"] = serve_run(torch, zig, tr, naive=False)
        log("serve %s batched: %s" % (name, json.dumps(run["batched"])))
        run["naive_per_request"] = serve_run(torch, zig, tr, naive=True)
        log("serve %s naive: %s" % (name, json.dumps(run["naive_per_request"])))
        out[name] = run
    return out


def moments_bench(torch, zig):
    """Fused generate-and-reduce (raw moment sums, no output written): the
    rate at 2^32 FP64 draws per distribution, and Appendix B's table of the
    raw moments X1..X5 from 10^12 draws of Exp(1) and N(0, 1) against the
    closed forms 1, 2, 6, 24, 120 and 0, 1, 0, 3, 0."""
    out = {}
    st = torch.cuda.current_stream()
    for name, dist, p0, p1 in [("exp", 0, 2.5, 0.0), ("normal", 1, -1.0, 3.0)]:
        n = 1 << 32
        zig.moments(dist, 0, n, 3, 0, p0, p1)  # warm-up at the measured size
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            zig.moments(dist, 0, n, 3, 0, p0, p1)
            b.record(st)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        out[name + "_2^32_f64"] = {"Gsamples/s": round(n / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 3),
                                   "runs": 5, "statistic": "median"}
    appb = {}
    for name, dist, want in [("exp", 0, [1, 2, 6, 24, 120]), ("normal", 1, [0, 1, 0, 3, 0])]:
        n = 10 ** 12
        t0 = time.perf_counter()
        s = zig.moments(dist, 0, n, 2014, 0, *((1.0, 0.0) if dist == 0 else (0.0, 1.0))).cpu().numpy()
        secs = time.perf_counter() - t0
        appb[name] = {"draws": n, "seconds": round(secs, 2), "moments": [float(v / n) for v in s],
                      "closed_form": want}
    out["appendix_b_1e12"] = appb
    return out


def traditional_ab(torch, zig):
    """The comparison of Table 1 on this GPU: the modified sampler and the
    traditional ziggurat on the headline fills (2^30 FP64, same streams,
    same tile/compaction/store kernel structure), each at its default
    shape and the traditional one also at its best of a few shapes."""
    out = torch.empty(N_C3, dtype=torch.float64, device="cuda")
    res = {}
    shapes = [(0, 0), (256, 8), (512, 4), (512, 2), (1024, 2), (512, 1)]
    for dist, name, seed, p0, p1 in [(0, "exp", 11, 2.5, 0.0), (1, "normal", 12, -1.0, 3.0)]:
        _, dd = timed_fills(torch, zig, [(lambda: zig.fill(out, dist, seed, 0, p0, p1), N_C3 * 8)], 10, 3)
        mod_ms = float(np.mean(dd))
        trad = {}
        for wg, spl in shapes:
            lt = zig.Launch(0, wg, spl, zig.LAUNCH_TRADITIONAL)
            _, dd = timed_fills(torch, zig, [(lambda: zig.fill(out, dist, seed, 0, p0, p1, launch=lt), N_C3 * 8)],
                                10, 3)
            trad["default" if wg == 0 else "%dx%d" % (wg, spl)] = round(float(np.mean(dd)), 4)
        best = min(trad, key=trad.get)
        mt = zig.zig_get_tables(dist, 256)
        tt = zig.zig_get_trad_tables(dist, 256)
        res[name] = {"modified_ms": round(mod_ms, 4), "traditional_ms": trad, "traditional_best": best,
                     "traditional_over_modified": round(trad[best] / mod_ms, 4),
                     "quick_exit": {"modified": mt["L"] / 256.0, "traditional": round(float(tt["k"].mean()), 5)}}
    del out
    torch.cuda.empty_cache()
    return res


def layers_ab(torch, zig):
    """Appendix D item 1 on this GPU: the headline fills (2^30, FP64 and
    FP32) with 1024 layers against 256, each at the default shape, the
    1024-layer kernels also at their best of a few shapes."""
    res = {}
    shapes = [(0, 0), (256, 8), (512, 4), (512, 2), (1024, 2)]
    for dtype, tname, esize in [(0, "f64", 8), (1, "f32", 4)]:
        out = torch.empty(N_C3, dtype=torch.float64 if dtype == 0 else torch.float32, device="cuda")
        for dist, name, seed, p0, p1 in [(0, "exp", 11, 2.5, 0.0), (1, "normal", 12, -1.0, 3.0)]:
            _, dd = timed_fills(torch, zig, [(lambda: zig.fill(out, dist, seed, 0, p0, p1), N_C3 * esize)], 10, 3)
            ms256 = float(np.mean(dd))
            wide = {}
            for wg, spl in shapes:
                lw = zig.Launch(1024, wg, spl, 0)
                _, dd = timed_fills(torch, zig, [(lambda: zig.fill(out, dist, seed, 0, p0, p1, launch=lw),
                                                  N_C3 * esize)], 10, 3)
                wide["default" if wg == 0 else "%dx%d" % (wg, spl)] = round(float(np.mean(dd)), 4)
            best = min(wide, key=wide.get)
            res["%s_%s" % (name, tname)] = {
                "ms_256_layers": round(ms256, 4), "ms_1024_layers": wide, "best_1024": best,
                "ratio_1024_over_256": round(wide[best] / ms256, 4),
                "slow_share": {"256": 1 - zig.zig_get_tables(dist, 256)["L"] / 256.0,
                               "1024": 1 - zig.zig_get_tables(dist, 1024)["L"] / 1024.0}}
        del out
        torch.cuda.empty_cache()
    return res


def autotune_report(zig):
    """Runs the autotuner on this device (cache in a temporary file) and
    reports, per (dist, dtype, size class), the chosen shape and its time
    against the built-in shape; the built-in table is restored after."""
    import tempfile
    d = tempfile.mkdtemp()
    path = os.path.join(d, "tune.json")
    t0 = time.perf_counter()
    zig.zig_autotune(path, zig.TUNE_FORCE)
    secs = time.perf_counter() - t0
    with open(path) as f:
        c = json.load(f)
    os.remove(path)
    os.rmdir(d)
    zig.zig_autotune_reset()
    rows = [{"dist": ["exp", "normal"][e["dist"]], "dtype": ["f64", "f32"][e["dtype"]], "n": e["n"],
             "shape": "%dx%d/%d" % (e["wg"], e["spl"], e["step_blocks"]), "us": e["us"],
             "builtin_us": e["default_us"]} for e in c["fill"]]
    return {"seconds": round(secs, 2), "fill": rows, "batch": c["batch"]}


def c2_bench(torch, zig):
    """2^28 N(0, 1) FP64 samples, seed 7, one launch: 3 warm-ups, the mean
    of 20 timed launches."""
    out = torch.empty(N_C2, dtype=torch.float64, device="cuda")
    _, dd = timed_fills(torch, zig, [(lambda: zig.fill_normal(out, 7, 0, 0.0, 1.0), N_C2 * 8)], 20, 3)
    ms = float(np.mean(dd))
    del out
    torch.cuda.empty_cache()
    return {"Gsamples/s": round(N_C2 / (ms * 1e-3) / 1e9, 2), "kernel_ms": round(ms, 4),
            "GB/s": round(N_C2 * 8 / (ms * 1e-3) / 1e9, 1)}


def slow_lane_stats(torch, zig, n=1 << 24):
    """Slow-lane and queue statistics from the trace build (per-output
    layer, first region, slow-stream words and density tests) over n
    outputs of each headline fill: the measured slow share against
    1 - L/i_max, slow-stream words and density tests per output (for the
    normal every box decision, squeezed or not), the share of
    64-block wave slices holding a slow output, and, per tile of the shape
    the headline size runs (2^30 outputs), the slow outputs a tile hands to
    its drain (mean, p99, max) and the drain's rounds (the longest
    slow-stream chain, in Philox blocks, among them)."""
    res = {}
    i32 = torch.int32
    for dist, name, seed, p0, p1 in [(0, "exp", 11, 2.5, 0.0), (1, "normal", 12, -1.0, 3.0)]:
        for dtype, tname in [(0, "f64"), (1, "f32")]:
            per_block = 2 if dtype == 0 else 4
            wg, spl, _ = zig.zig_tuned_shape(dist, dtype, N_C3)
            tile = wg * spl * per_block
            out = torch.empty(n, dtype=torch.float64 if dtype == 0 else torch.float32, device="cuda")
            layer, region, words, tests = (torch.empty(n, dtype=i32, device="cuda") for _ in range(4))
            zig.zig_fill_trace(dist, dtype, seed, 0, n, p0, p1, out.data_ptr(), layer.data_ptr(),
                               region.data_ptr(), words.data_ptr(), tests.data_ptr())
            torch.cuda.synchronize()
            slow = region >= 0
            blocks = torch.where(slow, (words + 1) // 2, torch.zeros_like(words))
            nt = n // tile
            per_tile = slow[:nt * tile].view(nt, tile).sum(1).double()
            rounds = blocks[:nt * tile].view(nt, tile).max(1).values.double()
            wave = slow[:(n // (64 * per_block)) * 64 * per_block].view(-1, 64 * per_block).any(1)
            res["%s_%s" % (name, tname)] = {
                "outputs": n,
                "slow_share": round(float(slow.double().mean()), 6),
                "slow_share_analytic": round(1 - zig.zig_get_tables(dist, 256)["L"] / 256.0, 6),
                "slow_words_per_output": round(float(words.double().sum()) / n, 5),
                "density_tests_per_output": round(float(tests.double().sum()) / n, 6),
                "wave_slices_with_slow_output": round(float(wave.double().mean()), 4),
                "tile": "%dx%d (%d outputs)" % (wg, spl, tile),
                "slow_per_tile": {"mean": round(float(per_tile.mean()), 2),
                                  "p99": float(torch.quantile(per_tile, 0.99)), "max": float(per_tile.max())},
                "drain_rounds_per_tile": {"mean": round(float(rounds.mean()), 3), "max": float(rounds.max())},
                "slow_stream_blocks_per_slow_output": round(float(blocks.double().sum() / slow.sum()), 4),
            }
            del out, layer, region, words, tests, slow, blocks
            torch.cuda.empty_cache()
    return res


def cpu_model():
    """The host CPU's model line from /proc/cpuinfo (empty if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline():
    """The oracle on the host cores, about 10-15 s of work: the first 2^32
    outputs of each headline stream on every core this process may run on
    (in chunks of 2^26, so host memory stays small), and the first 2^26 of
    each on one thread."""
    from oracle import oracle
    threads = max(1, len(os.sched_getaffinity(0)))
    chunk = 1 << 26

    def run(n, nthreads):
        t0 = time.perf_counter()
        for first in range(0, n, chunk):
            oracle.fill(0, 0, 11, first, chunk, 1.0 / 2.5, 0.0, threads=nthreads)
            oracle.fill(1, 0, 12, first, chunk, 3.0, -1.0, threads=nthreads)
        return time.perf_counter() - t0

    n_all, n_one = 1 << 32, 1 << 26  # per distribution
    t_all = run(n_all, threads)
    t_one = run(n_one, 1)
    return {
        "value": round(2 * n_all / t_all / 1e9, 5), "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
        "nproc": os.cpu_count(), "cpu_model": cpu_model(),
        "sample": "2^32 Exp(2.5) + 2^32 N(-1,3) FP64 outputs (indices 0..2^32-1 of the benchmark streams, "
                  "chunks of 2^26), %d threads over contiguous index ranges, %.1f s" % (threads, t_all),
        "single_thread": {"value": round(2 * n_one / t_one / 1e9, 5), "unit": "Gsamples/s",
                          "sample": "2^26 + 2^26 FP64 outputs, 1 thread, %.1f s" % t_one},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline step")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the 20k requests/s serving trace (the 200k/s trace runs 2 s)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 1 GiB (a kernel of known traffic, for scaling the "
                         "HBM byte counters of a profiler run)")
    ap.add_argument("--only", choices=["batch", "moments", "slow_lanes", "c2", "serving"],
                    help="run only this part and print it as the JSON line (for profiling one kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sampler shards by index range with no exchange step, "
              "so only --gpus 1 is run here", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1403_6870_amd import zig

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    log("device %s, %d CUs" % (props.name, props.multi_processor_count))
    zig.zig_build_tables(256)
    if args.only:
        part = {"batch": batch_bench, "moments": moments_bench, "slow_lanes": slow_lane_stats, "c2": c2_bench,
                "serving": lambda t, z: serve_bench(t, z, args.serve_seconds)}[args.only]
        print(json.dumps({"only": args.only, args.only: part(torch, zig)}), flush=True)
        return

    out_e = torch.empty(N_C3, dtype=torch.float64, device=dev)
    out_n = torch.empty(N_C3, dtype=torch.float64, device=dev)
    out_e.fill_(0.0)
    out_n.fill_(0.0)
    calls = [(lambda: zig.fill_exp(out_e, 11, 0, 2.5), N_C3 * 8),
             (lambda: zig.fill_normal(out_n, 12, 0, -1.0, 3.0), N_C3 * 8)]
    log("headline: %d steps of 2 x 2^30 FP64 fills" % args.steps)
    wall, durs = timed_fills(torch, zig, calls, args.steps, args.warmup)
    samples = 2 * N_C3 * args.steps
    value = samples / wall / 1e9
    d = np.array(durs)
    avg_ms = float(d[:, 1].mean())  # the normal fill, the dominant kernel
    bytes_per_launch = N_C3 * 8
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    log("headline: %.2f Gsamples/s; fill kernel exp %.3f ms, normal %.3f ms (%.0f GB/s)" %
        (value, d[:, 0].mean(), d[:, 1].mean(), achieved))
    # the store ceiling: a plain store kernel (torch's fill_) over the same
    # 8 GiB buffer, timed the same way
    _, ds = timed_fills(torch, zig, [(lambda: out_n.fill_(1.0), N_C3 * 8)], 10, 3)
    store_gbs = N_C3 * 8 / (float(np.mean(ds)) * 1e-3) / 1e9
    log("store ceiling (fill_ of 8 GiB): %.0f GB/s" % store_gbs)
    del out_e, out_n
    torch.cuda.empty_cache()
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
        torch.cuda.empty_cache()

    result = {
        "metric": "Gsamples/s FP64 exp+normal & % HBM-write roofline; batched p50/p99 latency",
        "value": round(value, 3), "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Philox4x32-10 streams)",
        "config": {"workload": "plain fill, FP64: 2^30 Exp(lambda=2.5) seed 11 + 2^30 N(mu=-1, sigma=3) seed 12, "
                               "256 layers, one launch each, output resident in HBM",
                   "samples_per_step": 2 * N_C3, "bytes_written_per_step": 2 * N_C3 * 8},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": TRAFFIC,
                     "kernel": "fill_kernel<normal, FP64> (the longer of the two launches of a step)",
                     "bytes_per_launch": bytes_per_launch,
                     "per_launch_ms": {"exp": round(float(d[:, 0].mean()), 4),
                                       "normal": round(float(d[:, 1].mean()), 4)},
                     "exp_fill_GB/s": round(bytes_per_launch / (float(d[:, 0].mean()) * 1e-3) / 1e9, 1),
                     "store_ceiling_GB/s": round(store_gbs, 1),
                     "frac_of_store_ceiling": round(achieved / store_gbs, 4)},
    }

    if not args.no_extra:
        extra = {}
        extra["normal_2^28_f64"] = c2_bench(torch, zig)
        # FP32 variants of the 2^30 fills
        o32 = torch.empty(N_C3, dtype=torch.float32, device=dev)
        for name, fn in [("exp_2^30_f32", lambda: zig.fill_exp(o32, 11, 0, 2.5)),
                         ("normal_2^30_f32", lambda: zig.fill_normal(o32, 12, 0, -1.0, 3.0))]:
            w, dd = timed_fills(torch, zig, [(fn, N_C3 * 4)], 10, 3)
            ms = float(np.mean(dd))
            extra[name] = {"Gsamples/s": round(N_C3 / (ms * 1e-3) / 1e9, 2), "kernel_ms": round(ms, 4),
                           "GB/s": round(N_C3 * 4 / (ms * 1e-3) / 1e9, 1)}
        del o32
        # the accelerated normal-overhang variant at the headline size
        out = torch.empty(N_C3, dtype=torch.float64, device=dev)
        lac = zig.Launch(0, 0, 0, zig.LAUNCH_NORMAL_ACCEL)
        w, dd = timed_fills(torch, zig, [(lambda: zig.fill(out, 1, 12, 0, -1.0, 3.0, launch=lac), N_C3 * 8)], 10, 3)
        ms = float(np.mean(dd))
        extra["normal_2^30_f64_accel_variant"] = {"Gsamples/s": round(N_C3 / (ms * 1e-3) / 1e9, 2),
                                                  "kernel_ms": round(ms, 4),
                                                  "GB/s": round(N_C3 * 8 / (ms * 1e-3) / 1e9, 1)}
        del out
        torch.cuda.empty_cache()
        log("extra: %s" % json.dumps(extra))
        result["other_configs"] = extra
        log("batched 4096-request workload")
        result["batch"] = batch_bench(torch, zig)
        log("batch: %s" % json.dumps(result["batch"]))
        if args.serve_seconds > 0:
            result["serving"] = serve_bench(torch, zig, args.serve_seconds)
        log("fused generate-and-reduce")
        result["moments"] = moments_bench(torch, zig)
        log("moments: %s" % json.dumps(result["moments"]))
        log("modified vs traditional ziggurat")
        result["traditional_ab"] = traditional_ab(torch, zig)
        log("traditional_ab: %s" % json.dumps(result["traditional_ab"]))
        log("slow-lane statistics (trace build)")
        result["slow_lanes"] = slow_lane_stats(torch, zig)
        log("slow_lanes: %s" % json.dumps(result["slow_lanes"]))
        log("1024 against 256 layers")
        result["layers_1024"] = layers_ab(torch, zig)
        log("layers_1024: %s" % json.dumps(result["layers_1024"]))
        log("autotuner")
        result["autotune"] = autotune_report(zig)
        log("autotune: %s" % json.dumps(result["autotune"]))

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline()
        log("cpu baseline: %s" % json.dumps(result["cpu_baseline"]))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
