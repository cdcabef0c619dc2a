"""The boundary from plain C: include/tabnet.h compiles as strict C99 (and C++17), and a C
program links against libtabnet.so and gets the documented status on an error path that
needs no GPU (a missing weight file is TABNET_E_IO, with a message and no handle)."""
import os
import shutil
import subprocess

import pytest

from paper_2510_19689_amd import tabnet as tb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_PROGRAM = r"""
#include <stdio.h>
#include "tabnet.h"

int main(void) {
    tabnet_handle* h = NULL;
    tabnet_status st = tabnet_load("/nonexistent/dir/model.tnw", TABNET_MXFP6_E3M2, 0, &h);
    const char* msg = tabnet_last_error();
    printf("abi %d status %d message %s\n", tabnet_abi_version(), (int)st, msg ? msg : "(none)");
    if (st != TABNET_E_IO || h != NULL || msg == NULL || msg[0] == '\0') return 1;
    /* argument errors are rejected before any device work */
    if (tabnet_forward(NULL, NULL, 0, NULL, NULL, NULL, NULL) != TABNET_E_INVALID) return 2;
    return 0;
}
"""


def test_header_is_strict_c_and_cxx():
    for comp, args in (("gcc", ["-std=c99", "-pedantic", "-x", "c"]), ("g++", ["-std=c++17", "-pedantic", "-x", "c++"])):
        exe = shutil.which(comp)
        if exe is None:
            pytest.skip(f"{comp} not available")
        for hdr in ("tabnet.h", "tabnet_internal.h"):
            r = subprocess.run([exe, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", *args,
                                os.path.join(ROOT, "include", hdr)], capture_output=True, text=True)
            assert r.returncode == 0, (comp, hdr, r.stderr)


def test_c_program_links_and_reports_errors(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    if not os.path.exists(tb.LIB_PATH):
        pytest.skip("libtabnet.so not built")
    libdir = os.path.dirname(os.path.abspath(tb.LIB_PATH))
    src = tmp_path / "use.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "use"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", f"-I{ROOT}/include", str(src),
                        "-o", str(exe), f"-L{libdir}", "-ltabnet", f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "status -4" in r.stdout


@pytest.mark.parametrize("prog", ["serve_load.c"])
def test_native_clients_build(tmp_path, prog):
    """The C clients under tests/native (the serving test's client and the load generator)
    compile as strict C99 and link against the library."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    if not os.path.exists(tb.LIB_PATH):
        pytest.skip("libtabnet.so not built")
    libdir = os.path.dirname(os.path.abspath(tb.LIB_PATH))
    r = subprocess.run([gcc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D_POSIX_C_SOURCE=199309L",
                        f"-I{ROOT}/include", os.path.join(ROOT, "tests", "native", prog), "-o", str(tmp_path / "a.out"),
                        f"-L{libdir}", "-ltabnet", f"-Wl,-rpath,{libdir}", "-pthread", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
