"""The serving API from a C program (tests/native/serve_load.c), on the GPU: several
threads submit requests back to back through include/tabnet.h; every request's rows equal
the same rows of every other request bit for bit, and every mask row is finite,
non-negative and sums to 1."""
import os
import shutil
import subprocess

import pytest

from paper_2510_19689_amd import synth, tabnet as tb

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("threads,requests,max_rows", [(1, 3000, 64), (4, 400, 4096)])
def test_c_client_serving(tmp_path, threads, requests, max_rows):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    if not os.path.exists(tb.LIB_PATH):
        pytest.fail("libtabnet.so not built")
    libdir = os.path.dirname(os.path.abspath(tb.LIB_PATH))
    exe = tmp_path / "serve_load"
    r = subprocess.run([gcc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", f"-I{ROOT}/include",
                        os.path.join(ROOT, "tests", "native", "serve_load.c"), "-o", str(exe), f"-L{libdir}",
                        "-ltabnet", f"-Wl,-rpath,{libdir}", "-pthread", "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    params, _ = synth.workload("adult108", rows=1)
    path = str(tmp_path / "adult108.tnw")
    synth.write_weights(params, path)
    print(f"case C client threads={threads} requests={requests} max_rows={max_rows}", flush=True)
    r = subprocess.run([str(exe), path, str(threads), str(requests), str(max_rows)], capture_output=True, text=True,
                       timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "failures 0" in r.stdout
