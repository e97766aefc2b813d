"""CPU: the oracle and the GPU-free host paths of libpitsbicg under
AddressSanitizer and UndefinedBehaviorSanitizer (with leak detection).

* tests/sanitize/oracle_driver.c runs every oracle entry point (1D IE and
  CN, 2D PR-ADI, the backward-Euler splitting, a rotating velocity; the
  FP32-fine form, a time-dependent operator, a separable source; every
  Algorithm 1 option and both parareal forms), built with gcc.
* tests/sanitize/host_driver.cpp runs the library's host code: pit_create on
  1D and 2D problems of every kernel family and its refusals, the table
  builders (line, column, velocity and per-slice tables), workspace sizing
  with sources and per-slice operators, the autotuner's candidate sizing,
  the batch engine's creation, and a randomized test of the request
  server's arena allocator against a model of the live ranges.  The library
  sources are compiled with the sanitizers on the host side only (device
  code is unchanged and never launched).
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_10148_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.slow


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...: rc {r.returncode}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def clean(r):
    out = r.stdout + r.stderr
    return "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fopenmp",
         "-ffp-contract=off", os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "pit_oracle.c"),
         "-o", exe, "-lm"])
    r = run([exe], env=ENV, timeout=600)
    assert "oracle driver: ok" in r.stdout and clean(r), r.stdout + r.stderr


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs.append(os.path.join(HERE, "host_driver.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run(["/opt/rocm/bin/hipcc", *flags, *san, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_driver")
    run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", *san, *objs, "-o", exe])
    r = run([exe], env=ENV, timeout=600)
    assert "host driver: ok" in r.stdout and clean(r), r.stdout + r.stderr
