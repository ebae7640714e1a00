"""CPU: the host-side code built with the address and undefined-behaviour
sanitizers and run.

* tests/host/plan_check.cpp includes the library's host planning
  (paper_1908_11740_amd/csrc/plan.hpp: the span-unit capacity bound the join
  workspace is sized from, the work-list check of the debug mode, the
  autotuner cache's line format) and checks the bound and the check against
  an independent walk of the classification's cutting rule.
* tests/host/oracle_check.c links the CPU oracle (oracle/sj_oracle.c) and
  runs its modes against each other on adversarial inputs, one and several
  OpenMP threads.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]


def _run(cmd, exe, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # the environment is left as it is; a library preloaded by the host
    # would come before the sanitizer runtime, which then must not insist
    # on being first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_bounds_and_checks_under_sanitizers(tmp_path):
    exe = tmp_path / "plan_check"
    out = _run(["g++", "-std=c++17", "-Wall", *SAN, "-o", str(exe),
                os.path.join(ROOT, "tests", "host", "plan_check.cpp")], exe, tmp_path)
    assert "plan checks passed" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_check"
    out = _run(["gcc", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-fopenmp", "-ffp-contract=off",
                *SAN, "-o", str(exe), os.path.join(ROOT, "tests", "host", "oracle_check.c"),
                os.path.join(ROOT, "oracle", "sj_oracle.c"), "-lm"], exe, tmp_path)
    assert "oracle checks passed" in out
