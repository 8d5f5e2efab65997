"""Host code under sanitizers (CPU only): the serving scheduler, driven on
its host fake backend by a multi-threaded stress program, and the
per-launch scratch-slot ring on a simulated device, under ThreadSanitizer
and under AddressSanitizer + UndefinedBehaviorSanitizer; the oracle's
entry points under AddressSanitizer + UBSan.  Each program is
built with g++/gcc from the committed sources (the library's device
objects are linked as built, uninstrumented) and must print "ok" with no
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1403_6870_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1403_6870_amd", "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
from paper_1403_6870_amd import build_lib  # noqa: E402  (source lists only; builds nothing on import)

HOST = list(build_lib.HOST_SRCS)
DEVICE_OBJS = [os.path.join(BUILD, s + ".o") for s in build_lib.HIP_SRCS]


def _run(cmd, **kw):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert p.returncode == 0, "%s\n%s" % (" ".join(cmd), p.stdout[-4000:])
    return p.stdout


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, san):
    if shutil.which("g++") is None or not all(os.path.exists(o) for o in DEVICE_OBJS):
        pytest.skip("needs g++ and the built device objects")
    flags = ["-O1", "-g", "-fsanitize=" + san, "-fno-omit-frame-pointer", "-std=gnu++17", "-fPIC",
             "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]
    objs = []
    srcs = [os.path.join(CSRC, s) for s in HOST] + [os.path.join(ROOT, "tests", "csrc", "server_stress.cpp")]
    procs = []
    for src in srcs:
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen(["g++"] + flags + ["-c", src, "-o", o], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    for p, src in zip(procs, srcs):
        out = p.communicate()[0]
        assert p.returncode == 0, "%s\n%s" % (src, out[-4000:])
    exe = str(tmp_path / "stress")
    _run(["g++", "-fsanitize=" + san, "-o", exe] + objs + DEVICE_OBJS +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lquadmath", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = _run([exe], env=env, timeout=600)
    assert out.strip().endswith("ok"), out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_slot_ring_under_sanitizer(tmp_path, san):
    """The per-launch scratch-slot ring (csrc/zig_ring.hpp) on a simulated
    device with in-order streams and events: 8 host threads, two of them
    sharing one stream, launch 24 000 kernels over 3 slots; no kernel may
    find its slot held by another launch or its counters non-zero.  (With
    the ring's wait removed the same program reports hundreds of
    violations.)"""
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "ring")
    _run(["g++", "-O1", "-g", "-fsanitize=" + san, "-fno-omit-frame-pointer", "-std=gnu++17",
          os.path.join(ROOT, "tests", "csrc", "ring_stress.cpp"), "-o", exe, "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = _run([exe], env=env, timeout=600)
    assert out.strip().endswith("ok"), out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out


def test_oracle_under_sanitizer(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-std=gnu11",
          "-ffp-contract=off", "-fno-fast-math", os.path.join(ROOT, "tests", "csrc", "oracle_sanitize.c"),
          os.path.join(ROOT, "oracle", "zig_oracle.c"), "-o", exe, "-lquadmath", "-lm", "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    out = _run([exe], env=env, timeout=600)
    assert out.strip().endswith("ok"), out[-4000:]
    assert "runtime error" not in out
