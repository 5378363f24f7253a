"""Sanitizer runs of the host code (CPU only; opt-in: PPST_SANITIZE=1).

* the library's host paths (parameter derivation, encoding and its threads,
  the binary128 bootstrapping plaintexts and their threads, the Chebyshev
  generators, argument checks) under AddressSanitizer + UndefinedBehavior-
  Sanitizer and under ThreadSanitizer: tests/test_abi_host.py against
  ``build.build_sanitized``'s library, its runtime preloaded;
* the oracle under AddressSanitizer + UndefinedBehaviorSanitizer (gcc): the
  oracle pins against ``ref.build_sanitized``'s library.

Each run is a child process (a sanitizer runtime has to be loaded first);
any report fails it (UB aborts, ASan and TSan halt on the first error).
The device code and the serving loop (which needs a GPU) are not covered.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2508_12093_amd"))

pytestmark = pytest.mark.skipif(os.environ.get("PPST_SANITIZE") != "1",
                                reason="sanitizer runs are opt-in (PPST_SANITIZE=1)")


def _run(env_extra, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env.pop("PPST_SANITIZE", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + tests,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=3000)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_library_host_code(kind):
    import build
    lib = build.build_sanitized(kind)
    opts = {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1",
            "TSAN_OPTIONS": "halt_on_error=1 report_signal_unsafe=0"}
    opts.update({"PPST_LIBRARY": lib, "LD_PRELOAD": build.sanitizer_runtime(kind)})
    _run(opts, ["tests/test_abi_host.py"])


def test_oracle():
    from oracle import ref
    out = os.path.join(ROOT, "_build", "san_oracle", "libckks_ref.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    ref.build_sanitized(out)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    _run({"ASAN_OPTIONS": "detect_leaks=0", "PPST_ORACLE_SO": out, "LD_PRELOAD": asan},
         ["tests/test_oracle_arith.py", "tests/test_oracle_ckks.py",
          "tests/test_oracle_sampling_encode.py", "tests/test_oracle_boot.py"])
