"""Build libppstat.so (HIP for gfx950) in-tree.

Every library source under csrc/ is compiled by hipcc for
--offload-arch=gfx950 and linked into paper_2508_12093_amd/libppstat.so; the
peak-rate microbenchmarks (csrc/probe.hip) go into libppstat_probe.so.
Objects go to _build/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libppstat.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["host_math.cpp", "eval.cpp", "stats.cpp", "server.cpp", "capi.cpp", "noalloc.cpp",
           "boot.cpp", "capi_boot.cpp", "ntt.hip", "kernels.hip"]
# host-only C++ built by g++ (binary128 arithmetic through libquadmath)
HOST_SOURCES = ["boot_host.cpp"]
CXX = os.environ.get("CXX_HOST", "g++")
HOST_FLAGS = ["-O2", "-fPIC", "-std=gnu++17", "-Wall", "-pthread"]

# peak-rate microbenchmarks for the roofline figures: a library of their own
PROBE_SOURCE = "probe.hip"
PROBE_OUT = os.path.join(HERE, "libppstat_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))
    return obj


def _compile_host(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [CXX] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed on %s:\n%s%s" % (CXX, src, r.stdout, r.stderr))
    return obj


def _link(objs, out, extra=()):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + list(objs) + list(extra)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + [PROBE_SOURCE]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        host = [ex.submit(_compile_host, h) for h in HOST_SOURCES]
        objs = list(ex.map(_compile, srcs))
        hobjs = [f.result() for f in host]
    _link(objs[:-1] + hobjs, OUT, ["-lpthread", "-lquadmath"])
    _link(objs[-1:], PROBE_OUT)
    if verbose:
        print("built", OUT, "and", PROBE_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
