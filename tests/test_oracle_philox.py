"""Pins of the oracle's uniform source: Philox4x32-10 against its published
known-answer vectors, and the stream layout (which block and word feeds
which output)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors(O):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert O.philox(ctr, key) == want


def _w64(x, hi):
    return (x[2] | (x[3] << 32)) if hi else (x[0] | (x[1] << 32))


@pytest.mark.parametrize("dist", [0, 1])
def test_fp64_fast_word_layout(O, dist):
    """Output n takes the fast word of block (n>>1, 0, 0): its low bits are
    the layer index and, on the fast path, its bits 11..63 times X_i 2^-53
    are the magnitude (normal sign from bit 10)."""
    seed = 0x1234_5678_9ABC_DEF1
    first = (1 << 33) - 5
    n = 64
    out, layer, region, words, tests = O.fill_trace(dist, 0, seed, first, n, 1.0, 0.0)
    tab = O.table_arrays(dist)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in range(n):
        idx = first + k
        m = idx >> 1
        x = O.philox([m & 0xFFFFFFFF, m >> 32, 0, 0], key)
        w = _w64(x, idx & 1)
        i = w & 255
        assert layer[k] == i
        if i < tab["L"]:
            assert region[k] == -1 and words[k] == 0
            mag = float(w >> 11) * tab["XS"][i]
            if dist == 1 and (w >> 10) & 1:
                mag = -mag
            assert out[k] == mag
        else:
            assert region[k] >= 0 and words[k] >= 3


@pytest.mark.parametrize("dist", [0, 1])
def test_fp32_fast_word_layout(O, dist):
    seed = 99
    first = 1001
    n = 64
    out, layer, region, words, tests = O.fill_trace(dist, 1, seed, first, n, 1.0, 0.0)
    tab = O.table_arrays(dist)
    for k in range(n):
        idx = first + k
        m = idx >> 2
        x = O.philox([m & 0xFFFFFFFF, m >> 32, 0, 1], [seed, 0])
        w = x[idx & 3]
        i = w & 255
        assert layer[k] == i
        if i < tab["L"]:
            if dist == 0:
                mag = np.float32(w >> 8) * tab["XS32"][i]
            else:
                mag = np.float32(w >> 9) * tab["XS32"][i]
                if (w >> 8) & 1:
                    mag = -mag
            assert out[k] == np.float32(mag)


def test_slow_stream_alias_word(O):
    """The first slow word of output n is word 0|1 of block (n, 0, 2); it
    selects the region through the alias table."""
    seed = 5
    n = 20000
    out, layer, region, words, tests = O.fill_trace(0, 0, seed, 0, n, 1.0)
    slow = np.nonzero(region >= 0)[0]
    assert len(slow) > 100
    for idx in slow[:50]:
        x = O.philox([int(idx), 0, 0, 2], [seed, 0])
        r = x[0] | (x[1] << 32)
        assert O.alias_draw(0, 256, r) == region[idx]


def test_split_and_threads_independent(O):
    """Outputs are a pure function of (seed, index): split calls and thread
    counts give the same bits."""
    for dist in (0, 1):
        for dtype in (0, 1):
            a = O.fill(dist, dtype, 3, 7, 10001, 1.5, 0.25, threads=1)
            b = np.concatenate([O.fill(dist, dtype, 3, 7, 4000, 1.5, 0.25, threads=3),
                                O.fill(dist, dtype, 3, 4007, 6001, 1.5, 0.25, threads=5)])
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
