"""The host-side plan code built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, no device code) and run over valid and invalid hierarchies: no sanitizer
report and the expected statuses.  CPU only; skipped where g++ or the sanitizer
runtimes are missing."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_plan_under_address_and_undefined_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "plan_driver")
    src = [os.path.join(HERE, "sanitize", "plan_driver.cpp"),
           os.path.join(ROOT, "paper_1410_0010_amd", "csrc", "plan.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe] + src
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0 and "sanitizer" in p.stdout.lower() and "cannot find" in p.stdout:
        pytest.skip("sanitizer runtimes not installed")
    assert p.returncode == 0, p.stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stdout
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, r.stdout
    assert "0 failure(s)" in r.stdout
