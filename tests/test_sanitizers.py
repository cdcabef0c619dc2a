"""The serving scheduler (host code) under ThreadSanitizer and AddressSanitizer+UBSan,
driven with the CPU stand-in executor (tests/native/serve_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_19689_amd", "csrc")
SRC = [os.path.join(ROOT, "tests", "native", "serve_driver.cpp"),
       os.path.join(CSRC, "tabnet_serve.cpp"), os.path.join(CSRC, "tabnet_serve_fake.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_serve_scheduler_sanitized(tmp_path, san):
    exe = str(tmp_path / "serve_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), *SRC, "-o", exe, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "runtime error" not in r.stderr, r.stderr
    assert "completed=160 bad=0" in r.stdout
    assert "wide completed=8 bad=0" in r.stdout
    assert "failed split request: bad=0" in r.stdout
