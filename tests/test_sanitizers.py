"""The host code (network simplex, oracle) under AddressSanitizer and
UndefinedBehaviorSanitizer, built with g++ into a plain executable (CPU only;
no GPU code is built with a sanitizer)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "tests", "native", "sanitize_driver.cpp"),
                           os.path.join(ROOT, "paper_2110_14734_amd", "csrc", "flow.cpp"),
                           os.path.join(ROOT, "oracle", "oracle.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "sanitized host checks ok" in r.stdout
