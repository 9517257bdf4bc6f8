"""AddressSanitizer / UndefinedBehaviorSanitizer runs of the CPU code.

The FP64 oracle is built with gcc and both sanitizers and driven by
tests/sanitize/oracle_driver.c; the library's host path (gjp_api.cpp: argument
validation, world -> grid conversion, the double-precision ray setup of the
sample count, trajectories, the launch-configuration cache, timing
bookkeeping) is compiled for the host only with the sanitizers and driven by
tests/sanitize/host_api_driver.cpp, whose stand-ins for the kernel launchers
abort if reached. Device code is never built with a sanitizer.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "gjp_oracle.c"),
          "-o", exe, "-lm"])
    r = _run([exe], env=ENV)
    assert "oracle driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_host_path_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "host_driver")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1609_00958_amd",
                                                                   "csrc")]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    objs = []
    for src in (os.path.join(ROOT, "paper_1609_00958_amd", "csrc", "gjp_api.cpp"),
                os.path.join(HERE, "host_api_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17",
              "-ffp-contract=off", *san, *inc, "-c", src, "-o", obj])
        objs.append(obj)
    _run([HIPCC, *san, *objs, "-o", exe])
    r = _run([exe], env=ENV)
    assert "host driver: ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
