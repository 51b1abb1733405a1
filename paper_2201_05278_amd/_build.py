"""Compile libsimwave_hip.so for gfx950 with hipcc (in-tree).

Each translation unit is compiled to an object in parallel (one unit per
stencil radius), then the objects are linked into the shared library.
"""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsimwave_hip.so")
SOURCES = ["plan.cpp", "api.cpp", "api64.cpp", "batch.cpp", "trace.cpp", "k_dispatch.cpp", "k_points.hip", "k_adjoint_vd.hip",
           "k_f64.hip"] + \
          [f"k_r{r}.hip" for r in range(1, 11)]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _compile(src, obj):
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
    return obj


def build(verbose=False, jobs=None):
    """Always recompiles; writes LIB atomically."""
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="swbuild") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(_compile, SOURCES, objs))
        tmp = LIB + ".tmp%d" % os.getpid()
        res = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                             capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
