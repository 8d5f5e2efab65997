"""Builds libzig.so (the sampler library) in-tree for gfx950.

Host sources are compiled with g++ (the table builder needs libquadmath),
the kernels with hipcc.  Device code is compiled without floating-point
contraction, so that only the explicit fma operations are fused, and
without packed FP32 instructions.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libzig.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SRCS = ["zig_tables.cpp", "zig_tune.cpp", "zig_api.cpp", "zig_batch.cpp", "zig_server.cpp"]
HIP_SRCS = ["zig_fill.hip", "zig_batch.hip", "zig_moments.hip", "zig_trad.hip", "zig_fill_wide.hip"]

HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-ffp-contract=off", "-Wall", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROCM, "include")]


def _run(cmd):
    p = subprocess.run(cmd, cwd=CSRC, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "is not a recognized feature for this target" not in l)
    if p.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose=False):
    """Compile every source and link libzig.so; always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HOST_SRCS:
        if os.path.exists(os.path.join(CSRC, s)):
            jobs.append(["g++"] + CXX_FLAGS + ["-c", s, "-o", os.path.join(BUILD, s + ".o")])
    for s in HIP_SRCS:
        if os.path.exists(os.path.join(CSRC, s)):
            jobs.append([os.path.join(ROCM, "bin", "hipcc")] + HIP_FLAGS + ["-c", s, "-o", os.path.join(BUILD, s + ".o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([os.path.join(ROCM, "bin", "hipcc"), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs +
         ["-lquadmath", "-Wl,--no-undefined"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
