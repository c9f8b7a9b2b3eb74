"""AddressSanitizer and UBSan builds of the host code, run on the CPU: the oracle
(``oracle/vor_oracle.c``, with gcc) and the host-side planning of a pipeline run
(``paper_1212_1095_amd/csrc/vor_plan.cpp``, host-only with hipcc; the sanitizer flags apply to
the host pass only).  The harnesses under ``tests/sanitize/`` drive ordinary inputs, boundary
sites, polygons and every input-error path; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"


def _build_and_run(cmd, exe, env_extra, expect):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, f"build failed:\n{r.stderr[-4000:]}"
    env = dict(os.environ, **env_extra)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and expect in r.stdout, (
        f"exit {r.returncode}\nstdout:\n{r.stdout[-2000:]}\nstderr:\n{r.stderr[-6000:]}")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_harness"
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "oracle", "vor_oracle.c"), os.path.join(HERE, "oracle_harness.c"),
           "-o", str(exe)]
    _build_and_run(cmd, exe, {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS":
                              "print_stacktrace=1:halt_on_error=1"}, "oracle harness ok")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_planning_under_asan_ubsan(tmp_path):
    exe = tmp_path / "plan_harness"
    csrc = os.path.join(ROOT, "paper_1212_1095_amd", "csrc")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(HERE, "plan_harness.cpp"), os.path.join(csrc, "vor_plan.cpp"),
           "-o", str(exe)]
    # the HIP runtime the executable links keeps allocations until exit: leaks not checked
    _build_and_run(cmd, exe, {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS":
                              "print_stacktrace=1:halt_on_error=1"}, "plan harness ok")
