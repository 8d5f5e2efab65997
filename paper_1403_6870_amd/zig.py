"""Python binding of libzig.so, the gfx950 modified-ziggurat sampler.

Argument marshalling only: every sample is produced by the library's HIP
kernels.  The functions named zig_* mirror the C ABI in include/zig.h one
to one (pointers are plain integers); fill_exp / fill_normal / fill /
fill_batch are conveniences that take torch tensors for device memory and
torch streams.  If the library has not been built, importing this module
raises ImportError: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzig.so")

ZIG_OK, ZIG_EINVAL, ZIG_ENOTABLES, ZIG_EHIP, ZIG_ENOMEM, ZIG_EBUSY, ZIG_ESTATE = range(7)
EXP, NORMAL = 0, 1
F64, F32 = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError("libzig.so is not built (run __graft_entry__.build() or paper_1403_6870_amd/build_lib.py)")

_lib = ctypes.CDLL(LIB_PATH)

u32, u64, i32, dbl, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p


class ZigError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("zig status %d: %s" % (status, msg))
        self.status = status


class TableView(ctypes.Structure):
    _fields_ = [("dist", u32), ("i_max", u32), ("b", u32), ("L", u32),
                ("X", ctypes.POINTER(dbl)), ("f", ctypes.POINTER(dbl)), ("XS", ctypes.POINTER(dbl)),
                ("XS32", ctypes.POINTER(ctypes.c_float)), ("W", ctypes.POINTER(dbl)), ("H", ctypes.POINTER(dbl)),
                ("q", ctypes.POINTER(u64)), ("T", ctypes.POINTER(u64)), ("alias", ctypes.POINTER(u32)),
                ("eps", dbl), ("K_eps", u64), ("X0", dbl), ("invX0", dbl),
                ("eps_cvx", dbl), ("del_ccv", dbl), ("K_cvx", u64), ("K_ccv", u64),
                ("sq_lo", ctypes.POINTER(u64)), ("sq_hi", ctypes.POINTER(u64))]


class TradView(ctypes.Structure):
    _fields_ = [("dist", u32), ("n", u32), ("b", u32), ("pad", u32),
                ("X", ctypes.POINTER(dbl)), ("f", ctypes.POINTER(dbl)), ("W", ctypes.POINTER(dbl)),
                ("WS", ctypes.POINTER(dbl)), ("k", ctypes.POINTER(dbl)), ("KQ", ctypes.POINTER(u64)),
                ("r", dbl), ("v", dbl), ("invr", dbl)]


class Launch(ctypes.Structure):
    _fields_ = [("i_max", u32), ("wg", u32), ("spl", u32), ("flags", u32)]


LAUNCH_NORMAL_ACCEL = 1
LAUNCH_TRADITIONAL = 2


class Request(ctypes.Structure):
    _fields_ = [("dist", u32), ("dtype", u32), ("seed", u64), ("first_index", u64), ("n", u64),
                ("p0", dbl), ("p1", dbl), ("out", vp)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("wg", u32), ("spl", u32), ("flags", u32)]


BATCH_NO_GRAPH = 1


class ServerCfg(ctypes.Structure):
    _fields_ = [("backend", u32), ("streams", u32), ("max_batch", u32), ("clients", u32), ("window_us", u32),
                ("fake_latency_us", u32), ("fake_fail_every", u32), ("pad", u32), ("cap_bytes", u64),
                ("seed_base", u64), ("arena", vp)]


class Spec(ctypes.Structure):
    _fields_ = [("dist", u32), ("dtype", u32), ("n", u64), ("p0", dbl), ("p1", dbl), ("t_arrival_ns", u64)]


class Completion(ctypes.Structure):
    _fields_ = [("status", i32), ("client", u32), ("dist", u32), ("dtype", u32), ("seed", u64),
                ("first_index", u64), ("n", u64), ("out", vp), ("batch_id", u64), ("batch_size", u32),
                ("pad", u32), ("t_arrival_ns", u64), ("t_submit_ns", u64), ("t_admit_ns", u64),
                ("t_launch_ns", u64), ("t_done_ns", u64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, u64) for k in ("batches", "requests", "samples", "failed_requests", "max_inflight_batches",
                                    "max_bytes_in_use", "bytes_in_use", "queued", "inflight_batches")]


class TraceItem(ctypes.Structure):
    _fields_ = [("client", u32), ("pad", u32), ("spec", Spec), ("copy_to", vp)]


BACKEND_DEVICE, BACKEND_HOST_FAKE = 0, 1
SUBMIT_NONBLOCK = 1
REPLAY_NAIVE = 1

# numpy views of the trace and completion arrays (same layout as the C structs)
TRACE_DTYPE = np.dtype([("client", np.uint32), ("pad", np.uint32), ("dist", np.uint32), ("dtype", np.uint32),
                        ("n", np.uint64), ("p0", np.float64), ("p1", np.float64), ("t_arrival_ns", np.uint64),
                        ("copy_to", np.uint64)])
COMPLETION_DTYPE = np.dtype([("status", np.int32), ("client", np.uint32), ("dist", np.uint32),
                             ("dtype", np.uint32), ("seed", np.uint64), ("first_index", np.uint64),
                             ("n", np.uint64), ("out", np.uint64), ("batch_id", np.uint64),
                             ("batch_size", np.uint32), ("pad", np.uint32), ("t_arrival_ns", np.uint64),
                             ("t_submit_ns", np.uint64), ("t_admit_ns", np.uint64), ("t_launch_ns", np.uint64),
                             ("t_done_ns", np.uint64)])
assert TRACE_DTYPE.itemsize == ctypes.sizeof(TraceItem)
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(Completion)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_build = _sig("zig_build_tables", i32, [u32])
_get = _sig("zig_get_tables", i32, [u32, u32, ctypes.POINTER(TableView)])
_get_trad = _sig("zig_get_trad_tables", i32, [u32, u32, ctypes.POINTER(TradView)])
_fill_exp = _sig("zig_fill_exp", i32, [u64, u64, u64, u32, dbl, vp, vp])
_fill_normal = _sig("zig_fill_normal", i32, [u64, u64, u64, u32, dbl, dbl, vp, vp])
_fill = _sig("zig_fill", i32, [u32, u32, u64, u64, u64, dbl, dbl, vp, vp, ctypes.POINTER(Launch)])
_fill_trace = _sig("zig_fill_trace", i32, [u32, u32, u64, u64, u64, dbl, dbl, vp, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(Launch)])
_fill_batch = _sig("zig_fill_batch", i32, [ctypes.POINTER(Request), u32, vp])
_fill_batch_ex = _sig("zig_fill_batch_ex", i32, [ctypes.POINTER(Request), u32, vp, ctypes.POINTER(BatchOpts)])
_fill_each = _sig("zig_fill_each", i32, [ctypes.POINTER(Request), u32, vp])
_autotune = _sig("zig_autotune", i32, [ctypes.c_char_p, u32])
_tuned_shape = _sig("zig_tuned_shape", i32, [u32, u32, u64, ctypes.POINTER(Launch), ctypes.POINTER(u32)])
_tuned_batch_shape = _sig("zig_tuned_batch_shape", i32, [ctypes.POINTER(BatchOpts)])
_autotune_reset = _sig("zig_autotune_reset", i32, [])
TUNE_LOAD, TUNE_FORCE = 1, 2
_srv_p = ctypes.c_void_p
_server_now = _sig("zig_server_now_ns", u64, [])
_server_create = _sig("zig_server_create", i32, [ctypes.POINTER(ServerCfg), ctypes.POINTER(_srv_p)])
_server_submit = _sig("zig_server_submit", i32, [_srv_p, u32, ctypes.POINTER(Spec), u32, ctypes.POINTER(u64)])
_server_wait = _sig("zig_server_wait", i32, [_srv_p, u64, ctypes.c_int64, ctypes.POINTER(Completion)])
_server_release = _sig("zig_server_release", i32, [_srv_p, u64])
_server_drop = _sig("zig_server_drop_client", i32, [_srv_p, u32, ctypes.POINTER(u64)])
_server_counters = _sig("zig_server_counters", i32, [_srv_p, vp, u32])
_server_set_counters = _sig("zig_server_set_counters", i32, [_srv_p, vp, u32])
_server_stats = _sig("zig_server_stats_get", i32, [_srv_p, ctypes.POINTER(ServerStats)])
_server_replay = _sig("zig_server_replay", i32, [_srv_p, vp, u64, u32, vp])
_server_destroy = _sig("zig_server_destroy", i32, [_srv_p])
_moments = _sig("zig_moments", i32, [u32, u32, u64, u64, u64, dbl, dbl, vp, vp, ctypes.POINTER(Launch)])
_moments_noalloc = _sig("zig_moments_noalloc", i32, [u32, u32, u64, u64, u64, dbl, dbl, vp, vp,
                                                     ctypes.POINTER(Launch)])
_last_error = _sig("zig_last_error", ctypes.c_char_p, [])
_version = _sig("zig_version", ctypes.c_char_p, [])

EXPORTS = ["zig_build_tables", "zig_get_tables", "zig_get_trad_tables", "zig_fill_exp", "zig_fill_normal", "zig_fill",
           "zig_fill_trace", "zig_fill_batch", "zig_fill_batch_ex", "zig_fill_each", "zig_moments", "zig_autotune",
           "zig_tuned_shape", "zig_tuned_batch_shape", "zig_autotune_reset", "zig_server_now_ns", "zig_server_create",
           "zig_server_submit", "zig_server_wait", "zig_server_release", "zig_server_drop_client",
           "zig_server_counters", "zig_server_set_counters", "zig_server_stats_get", "zig_server_replay",
           "zig_server_destroy", "zig_last_error", "zig_version"]


def zig_last_error():
    return _last_error().decode()


def zig_version():
    return _version().decode()


def _check(status):
    if status != ZIG_OK:
        raise ZigError(status, zig_last_error())


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, Launch):
        return ctypes.byref(launch)
    return ctypes.byref(Launch(launch.get("i_max", 0), launch.get("wg", 0), launch.get("spl", 0),
                               launch.get("flags", 0)))


def zig_build_tables(i_max=256):
    _check(_build(i_max))


def zig_get_tables(dist, i_max=256):
    v = TableView()
    _check(_get(dist, i_max, ctypes.byref(v)))
    L, im = v.L, v.i_max
    arr = lambda p, k, dt: np.ctypeslib.as_array(p, shape=(k,)).astype(dt).copy()
    return {
        "dist": v.dist, "i_max": im, "b": v.b, "L": L,
        "X": arr(v.X, L + 1, np.float64), "f": arr(v.f, L + 1, np.float64),
        "XS": arr(v.XS, im, np.float64), "XS32": arr(v.XS32, im, np.float32),
        "W": arr(v.W, L + 1, np.float64), "H": arr(v.H, L + 1, np.float64),
        "q": arr(v.q, L + 1, np.uint64), "T": arr(v.T, im, np.uint64), "A": arr(v.alias, im, np.uint32),
        "eps": v.eps, "K_eps": int(v.K_eps), "X0": v.X0, "invX0": v.invX0,
        "eps_cvx": v.eps_cvx, "del_ccv": v.del_ccv, "K_cvx": int(v.K_cvx), "K_ccv": int(v.K_ccv),
        "sq_lo": arr(v.sq_lo, L + 1, np.uint64) if v.sq_lo else None,
        "sq_hi": arr(v.sq_hi, L + 1, np.uint64) if v.sq_hi else None,
    }


def zig_get_trad_tables(dist, i_max=256):
    v = TradView()
    _check(_get_trad(dist, i_max, ctypes.byref(v)))
    n = v.n
    arr = lambda p, dt: np.ctypeslib.as_array(p, shape=(n,)).astype(dt).copy()
    return {
        "dist": v.dist, "n": n, "b": v.b,
        "X": arr(v.X, np.float64), "f": arr(v.f, np.float64), "W": arr(v.W, np.float64),
        "WS": arr(v.WS, np.float64), "k": arr(v.k, np.float64), "KQ": arr(v.KQ, np.uint64),
        "r": v.r, "v": v.v, "invr": v.invr,
    }


def zig_fill_exp(seed, first_index, n, dtype, lam, out_ptr, stream_ptr=None):
    _check(_fill_exp(seed, first_index, n, dtype, lam, out_ptr, stream_ptr))


def zig_fill_normal(seed, first_index, n, dtype, mu, sigma, out_ptr, stream_ptr=None):
    _check(_fill_normal(seed, first_index, n, dtype, mu, sigma, out_ptr, stream_ptr))


def zig_fill(dist, dtype, seed, first_index, n, p0, p1, out_ptr, stream_ptr=None, launch=None):
    _check(_fill(dist, dtype, seed, first_index, n, p0, p1, out_ptr, stream_ptr, _launch(launch)))


def zig_fill_trace(dist, dtype, seed, first_index, n, p0, p1, out_ptr, layer_ptr, region_ptr, words_ptr, tests_ptr,
                   stream_ptr=None, launch=None):
    _check(_fill_trace(dist, dtype, seed, first_index, n, p0, p1, out_ptr, layer_ptr, region_ptr, words_ptr,
                       tests_ptr, stream_ptr, _launch(launch)))


def zig_fill_batch(reqs, stream_ptr=None, opts=None):
    """reqs: a ctypes array of Request (or a sequence of Request)."""
    if not isinstance(reqs, ctypes.Array):
        reqs = (Request * len(reqs))(*reqs)
    if opts is None:
        _check(_fill_batch(reqs, len(reqs), stream_ptr))
    else:
        if not isinstance(opts, BatchOpts):
            opts = BatchOpts(opts.get("wg", 0), opts.get("spl", 0), opts.get("flags", 0))
        _check(_fill_batch_ex(reqs, len(reqs), stream_ptr, ctypes.byref(opts)))


def zig_fill_each(reqs, stream_ptr=None):
    if not isinstance(reqs, ctypes.Array):
        reqs = (Request * len(reqs))(*reqs)
    _check(_fill_each(reqs, len(reqs), stream_ptr))


def zig_moments(dist, dtype, seed, first_index, n, p0, p1, sums_ptr, stream_ptr=None, launch=None):
    _check(_moments(dist, dtype, seed, first_index, n, p0, p1, sums_ptr, stream_ptr, _launch(launch)))


def zig_moments_noalloc(dist, dtype, seed, first_index, n, p0, p1, sums_ptr, stream_ptr=None, launch=None):
    _check(_moments_noalloc(dist, dtype, seed, first_index, n, p0, p1, sums_ptr, stream_ptr, _launch(launch)))


def zig_autotune(cache_path=None, flags=0):
    _check(_autotune(cache_path.encode() if cache_path else None, flags))


def zig_tuned_shape(dist, dtype, n):
    """(wg, spl, step_blocks) a fill of (dist, dtype, n) uses."""
    la, step = Launch(), u32()
    _check(_tuned_shape(dist, dtype, n, ctypes.byref(la), ctypes.byref(step)))
    return la.wg, la.spl, step.value


def zig_tuned_batch_shape():
    o = BatchOpts()
    _check(_tuned_batch_shape(ctypes.byref(o)))
    return o.wg, o.spl


def zig_autotune_reset():
    _check(_autotune_reset())


def zig_server_now_ns():
    return int(_server_now())


class Server:
    """Owner of a zig_server handle (the serving loop); methods mirror the
    zig_server_* calls.  Use as a context manager or call close()."""

    def __init__(self, cap_bytes, backend=BACKEND_DEVICE, streams=0, max_batch=0, clients=0, window_us=0,
                 seed_base=0, arena_ptr=None, fake_latency_us=0, fake_fail_every=0):
        self.cfg = ServerCfg(backend, streams, max_batch, clients, window_us, fake_latency_us, fake_fail_every, 0,
                             cap_bytes, seed_base, arena_ptr)
        self.clients = clients or 64
        h = _srv_p()
        _check(_server_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h

    def _handle(self):
        if self._h is None:
            raise ZigError(ZIG_ESTATE, "server closed")
        return self._h

    def submit(self, client, dist, dtype, n, p0=1.0, p1=1.0, t_arrival_ns=0, nonblock=False):
        spec = Spec(dist, dtype, n, p0, p1, t_arrival_ns)
        t = u64()
        _check(_server_submit(self._handle(), client, ctypes.byref(spec), SUBMIT_NONBLOCK if nonblock else 0,
                              ctypes.byref(t)))
        return t.value

    def wait(self, ticket, timeout_us=-1):
        """Completion record of a request; raises ZigError if it failed,
        was cancelled or the wait timed out."""
        c = Completion()
        _check(_server_wait(self._handle(), ticket, timeout_us, ctypes.byref(c)))
        return c

    def poll(self, ticket, timeout_us=-1):
        """(status, completion) without raising on the request's status."""
        c = Completion()
        st = _server_wait(self._handle(), ticket, timeout_us, ctypes.byref(c))
        return st, c

    def release(self, ticket):
        _check(_server_release(self._handle(), ticket))

    def drop_client(self, client):
        n = u64()
        _check(_server_drop(self._handle(), client, ctypes.byref(n)))
        return n.value

    def counters(self, count=None):
        count = self.clients if count is None else count
        a = np.zeros(count, dtype=np.uint64)
        _check(_server_counters(self._handle(), a.ctypes.data, count))
        return a

    def set_counters(self, values):
        a = np.ascontiguousarray(values, dtype=np.uint64)
        _check(_server_set_counters(self._handle(), a.ctypes.data, len(a)))

    def stats(self):
        st = ServerStats()
        _check(_server_stats(self._handle(), ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def replay(self, trace, naive=False):
        """trace: numpy array of TRACE_DTYPE (t_arrival_ns = offset from the
        start); returns the COMPLETION_DTYPE array."""
        trace = np.ascontiguousarray(trace, dtype=TRACE_DTYPE)
        out = np.zeros(len(trace), dtype=COMPLETION_DTYPE)
        st = _server_replay(self._handle(), trace.ctypes.data, len(trace), REPLAY_NAIVE if naive else 0,
                            out.ctypes.data)
        if st != ZIG_OK:
            raise ZigError(st, zig_last_error())
        return out

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(_server_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- torch conveniences -------------------------------------------------

def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("output tensor must be float64 or float32")


def _check_out(out):
    if not out.is_cuda or not out.is_contiguous():
        raise ValueError("output must be a contiguous device tensor")


def fill(out, dist, seed, first_index=0, p0=1.0, p1=1.0, launch=None, stream=None):
    """Fill a contiguous float64/float32 device tensor with samples
    first_index .. first_index + numel - 1; dist EXP (p0 = lambda) or
    NORMAL (p0 = mu, p1 = sigma)."""
    _check_out(out)
    zig_fill(dist, _dtype_code(out), seed, first_index, out.numel(), p0, p1, out.data_ptr(), _stream_ptr(stream),
             launch)
    return out


def fill_exp(out, seed, first_index=0, lam=1.0, stream=None):
    _check_out(out)
    zig_fill_exp(seed, first_index, out.numel(), _dtype_code(out), lam, out.data_ptr(), _stream_ptr(stream))
    return out


def fill_normal(out, seed, first_index=0, mu=0.0, sigma=1.0, stream=None):
    _check_out(out)
    zig_fill_normal(seed, first_index, out.numel(), _dtype_code(out), mu, sigma, out.data_ptr(), _stream_ptr(stream))
    return out


def fill_trace(out, dist, seed, first_index=0, p0=1.0, p1=1.0, launch=None, stream=None):
    """Debug fill that also returns per-output (layer, region, words,
    tests) device tensors."""
    import torch
    _check_out(out)
    n = out.numel()
    layer = torch.empty(n, dtype=torch.int32, device=out.device)
    region = torch.empty(n, dtype=torch.int32, device=out.device)
    words = torch.empty(n, dtype=torch.int32, device=out.device)
    tests = torch.empty(n, dtype=torch.int32, device=out.device)
    zig_fill_trace(dist, _dtype_code(out), seed, first_index, n, p0, p1, out.data_ptr(), layer.data_ptr(),
                   region.data_ptr(), words.data_ptr(), tests.data_ptr(), _stream_ptr(stream), launch)
    return out, layer, region, words, tests


def moments(dist, dtype, n, seed, first_index=0, p0=1.0, p1=1.0, stream=None, i_max=0, spl=0, accel=False):
    """Raw moment sums S1..S5 of the n outputs (dtype F64 or F32) as a
    float64 device tensor of 5 elements; nothing else is written."""
    import torch
    sums = torch.empty(5, dtype=torch.float64, device="cuda")
    la = None
    if i_max or spl or accel:
        la = Launch(i_max, 256 if spl else 0, spl, LAUNCH_NORMAL_ACCEL if accel else 0)
    zig_moments(dist, dtype, seed, first_index, n, p0, p1, sums.data_ptr(), _stream_ptr(stream), la)
    return sums


def fill_batch(items, stream=None, opts=None):
    """items: sequence of (out_tensor, dist, seed, first_index, p0, p1); all
    filled by one batched launch."""
    reqs = (Request * len(items))()
    for k, (out, dist, seed, first, p0, p1) in enumerate(items):
        _check_out(out)
        reqs[k] = Request(dist, _dtype_code(out), seed, first, out.numel(), p0, p1, out.data_ptr())
    zig_fill_batch(reqs, _stream_ptr(stream), opts)
