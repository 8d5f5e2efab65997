"""GPU tests of the autotuner: it writes a complete cache for this device,
fills and batches use the tuned shapes, the outputs of tuned shapes are
bit-identical to the built-in ones (the shape never changes a sample), a
cache is reloaded only on a matching device, and a reset restores the
built-in table."""
import json

import numpy as np
import pytest

from helpers import EXP, F32, F64, NORMAL

pytestmark = pytest.mark.gpu

FILL_SHAPES = {(w, s) for w in (64, 128, 256, 512, 1024) for s in (1, 2, 4, 8) if w * s <= 2048} | {(256, 7), (256, 10)}
BATCH_SHAPES = {(64, 4), (128, 4), (128, 8), (256, 2), (256, 4), (512, 2)}


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_1403_6870_amd import zig
    assert torch.cuda.is_available()
    return torch, zig


@pytest.fixture(scope="module")
def tuned(env, tmp_path_factory):
    torch, zig = env
    path = str(tmp_path_factory.mktemp("tune") / "cache.json")
    builtin = {(d, t, n): zig.zig_tuned_shape(d, t, n) for d in (0, 1) for t in (0, 1)
               for n in (1000, 1 << 20, 1 << 24, 1 << 30)}
    zig.zig_autotune(path, zig.TUNE_FORCE)
    yield path, builtin
    zig.zig_autotune_reset()


def test_cache_is_complete(env, tuned):
    torch, zig = env
    path, _ = tuned
    with open(path) as f:
        c = json.load(f)
    props = torch.cuda.get_device_properties(0)
    assert c["format"] == "zig-autotune-1" and c["cus"] == props.multi_processor_count
    keys = {(e["dist"], e["dtype"], e["class"]) for e in c["fill"]}
    assert keys == {(d, t, k) for d in (0, 1) for t in (0, 1) for k in range(4)}
    for e in c["fill"]:
        assert (e["wg"], e["spl"]) in FILL_SHAPES
        assert e["us"] > 0 and e["us"] <= e["default_us"] * 1.0001
        assert zig.zig_tuned_shape(e["dist"], e["dtype"], e["n"]) == (e["wg"], e["spl"], e["step_blocks"])
    assert (c["batch"]["wg"], c["batch"]["spl"]) in BATCH_SHAPES
    assert zig.zig_tuned_batch_shape() == (c["batch"]["wg"], c["batch"]["spl"])


@pytest.mark.parametrize("dist,dtype,n", [(EXP, F64, 70001), (NORMAL, F32, 3 * 2 ** 20 + 5),
                                          (NORMAL, F64, 2 ** 22 + 3), (EXP, F32, 2 ** 26 + 1)])
def test_tuned_outputs_equal_builtin(env, tuned, dist, dtype, n):
    torch, zig = env
    _, builtin = tuned
    dt = torch.float64 if dtype == F64 else torch.float32
    a = torch.empty(n, dtype=dt, device="cuda")
    b = torch.empty(n, dtype=dt, device="cuda")
    zig.fill(a, dist, 99, 12345, 1.7, 0.6)  # tuned shape
    wg, spl, _ = builtin[(dist, dtype, 1 << 30)]
    zig.fill(b, dist, 99, 12345, 1.7, 0.6, launch=zig.Launch(256, wg, spl))
    assert torch.equal(a, b)


def test_cache_reload_and_mismatch(env, tuned, tmp_path):
    torch, zig = env
    path, builtin = tuned
    want = {k: zig.zig_tuned_shape(*k) for k in builtin}
    zig.zig_autotune_reset()
    assert {k: zig.zig_tuned_shape(*k) for k in builtin} == builtin
    zig.zig_autotune(path, zig.TUNE_LOAD)
    assert {k: zig.zig_tuned_shape(*k) for k in builtin} == want
    # a cache written for another compute-unit count is not used
    other = tmp_path / "other.json"
    text = open(path).read()
    cus = json.loads(text)["cus"]
    other.write_text(text.replace('"cus": %d,' % cus, '"cus": %d,' % (cus + 1)))
    with pytest.raises(zig.ZigError) as e:
        zig.zig_autotune(str(other), zig.TUNE_LOAD)
    assert e.value.status == zig.ZIG_ESTATE and "another device" in str(e.value)
    with pytest.raises(zig.ZigError) as e:
        zig.zig_autotune(str(tmp_path / "missing.json"), zig.TUNE_LOAD)
    assert e.value.status == zig.ZIG_ESTATE
    # a damaged cache is refused as a whole
    bad = tmp_path / "bad.json"
    bad.write_text(text.replace('"wg": ', '"wg": 3', 1))
    with pytest.raises(zig.ZigError):
        zig.zig_autotune(str(bad), zig.TUNE_LOAD)
    assert {k: zig.zig_tuned_shape(*k) for k in builtin} == want


def test_batch_with_tuned_shape_equals_single(env, tuned):
    torch, zig = env
    rng = np.random.default_rng(3)
    items = []
    for k in range(300):
        n = int(2 ** (16 * rng.random()))
        dt = torch.float64 if k % 2 else torch.float32
        items.append((torch.empty(n, dtype=dt, device="cuda"), k % 3 == 0, k, int(rng.integers(0, 99)), 1.3, 0.7))
    zig.fill_batch([(o, int(d), s, f, p0, p1) for (o, d, s, f, p0, p1) in items])
    for o, d, s, f, p0, p1 in items[::7]:
        w = torch.empty_like(o)
        zig.fill(w, int(d), s, f, p0, p1)
        assert torch.equal(o, w)
