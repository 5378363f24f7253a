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


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-x", "hip"] + FLAGS + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))
    return obj


def _compile_host(src: str, build_dir: str = BUILD, cxx: str = CXX, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [cxx] + HOST_FLAGS + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s failed on %s:\n%s%s" % (cxx, src, r.stdout, r.stderr))
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


# Sanitizer builds of the host code (the device code is built as usual):
# "address" = AddressSanitizer + UndefinedBehaviorSanitizer, "thread" =
# ThreadSanitizer.  Every flag goes to the host pass only (-Xarch_host); the
# binary128 file is built with the same clang so that one sanitizer runtime
# serves the whole library.  Load the result with that runtime preloaded
# (sanitizer_runtime(kind)); tests/test_sanitizers.py runs the CPU suite's
# host-only library tests against it.
SAN_FLAGS = {
    "address": ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"],
    "thread": ["-fsanitize=thread"],
}
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def _gcc_private_include() -> list:
    """gcc's own include directory (quadmath.h lives there), searched after
    clang's headers."""
    r = subprocess.run(["gcc", "-print-file-name=include"], capture_output=True, text=True)
    d = r.stdout.strip()
    return ["-idirafter", d] if d and os.path.isdir(d) else []


def sanitizer_runtime(kind: str) -> str:
    lib = {"address": "libclang_rt.asan-x86_64.so", "thread": "libclang_rt.tsan-x86_64.so"}[kind]
    base = "/opt/rocm/llvm/lib/clang"
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", lib)
        if os.path.exists(p):
            return p
    raise RuntimeError("no %s runtime under %s" % (kind, base))


def build_sanitized(kind: str, verbose: bool = False) -> str:
    flags = SAN_FLAGS[kind]
    bdir = os.path.join(BUILD, "san_" + kind)
    out = os.path.join(bdir, "libppstat.so")
    os.makedirs(bdir, exist_ok=True)
    host_extra = []
    for f in flags:
        host_extra += ["-Xarch_host", f]
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        host = [ex.submit(_compile_host, h, bdir, CLANGXX, flags + _gcc_private_include())
                for h in HOST_SOURCES]
        objs = list(ex.map(lambda src: _compile(src, bdir, host_extra), SOURCES))
        hobjs = [f.result() for f in host]
    # the sanitizer symbols stay undefined in the shared object and resolve
    # to the preloaded runtime
    _link(objs + hobjs, out, ["-lpthread", "-lquadmath"])
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--sanitize":
        build_sanitized(sys.argv[2], verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
