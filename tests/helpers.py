"""Shared test helpers: library fills on the GPU, oracle fills on the CPU,
and the parity comparison."""
import os

import numpy as np

EXP, NORMAL = 0, 1
F64, F32 = 0, 1
THREADS = max(1, min(16, os.cpu_count() or 1))


def oracle_fill(O, dist, dtype, seed, first, n, p0, p1, i_max=256, threads=THREADS):
    """Oracle samples with the library's parameter convention (exp: p0 =
    lambda; normal: p0 = mu, p1 = sigma)."""
    if dist == EXP:
        return O.fill(EXP, dtype, seed, first, n, 1.0 / p0, 0.0, threads=threads, i_max=i_max)
    return O.fill(NORMAL, dtype, seed, first, n, p1, p0, threads=threads, i_max=i_max)


def gpu_fill(dist, dtype, seed, first, n, p0, p1, launch=None, out=None):
    import torch

    from paper_1403_6870_amd import zig
    if out is None:
        out = torch.empty(n, dtype=torch.float64 if dtype == F64 else torch.float32, device="cuda")
    zig.fill(out, dist, seed, first, p0, p1, launch=launch)
    return out


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _ordered(a):
    """Map floats to integers whose differences count representable
    values in between (-0 and +0 both map to 0)."""
    if a.dtype == np.float64:
        i = a.view(np.int64)
        return np.where(i < 0, np.int64(-(2 ** 63)) - i, i)
    i = a.view(np.int32).astype(np.int64)
    return np.where(i < 0, -(i + 2 ** 31), i)


def ulp_distance(a, b):
    """Distance in units in the last place between same-dtype float arrays."""
    return np.abs(_ordered(a) - _ordered(b))


def parity(got, want, max_ulp, exact=None):
    """Element-wise parity: returns (n_not_bit_identical, max ulp) and
    asserts the ulp bound; where the boolean mask `exact` is set (outputs
    on the fast path) the values must be bit-identical."""
    assert got.shape == want.shape and got.dtype == want.dtype
    it = np.int64 if got.dtype == np.float64 else np.int32
    diff = got.view(it) != want.view(it)
    if exact is not None:
        bad = int(np.count_nonzero(diff & exact))
        assert bad == 0, "%d fast-path outputs are not bit-identical" % bad
    nd = int(np.count_nonzero(diff))
    mu = 0
    if nd:
        mu = int(ulp_distance(got[diff], want[diff]).max())
    assert mu <= max_ulp, "%d outputs differ, max %d ulp (allowed %d)" % (nd, mu, max_ulp)
    return nd, mu
