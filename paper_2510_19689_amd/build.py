"""Build libtabnet.so (HIP for gfx950) in-tree.

    python -m paper_2510_19689_amd.build          # or build() from Python

Every source is compiled by hipcc for gfx950 only.  Packed-FP32 VALU instructions are
disabled in device code (-packed-fp32-ops off); the host pass warns that it does not
know the feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtabnet.so")
ARCH = "gfx950"

TEST_LIB = os.path.join(HERE, "libtabnet_test.so")

# libtabnet.so: the product.  libtabnet_test.so: the same code plus the host-only test
# hooks (include/tabnet_internal.h) and the serving runtime's CPU stand-in device.
SOURCES = [
    "tabnet_kernel.hip",
    "tabnet_generic_fp32.hip",
    "tabnet_generic_bf16.hip",
    "tabnet_generic_fp8w.hip",
    "tabnet_generic_fp8.hip",
    "tabnet_generic_int8.hip",
    "tabnet_generic_fp32_raw.hip",
    "tabnet_generic_bf16_raw.hip",
    "tabnet_stats.hip",
    "tabnet_pack.cpp",
    "tabnet_api.cpp",
    "tabnet_serve.cpp",
    "tabnet_serve_exec.cpp",
]
TEST_SOURCES = [
    "tabnet_hooks.cpp",
    "tabnet_serve_fake.cpp",
]

COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libtabnet")


def _compile(src: str, obj: str, defines=()) -> None:
    cmd = [hipcc(), *COMMON, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noise and os.environ.get("TABNET_BUILD_VERBOSE"):
        sys.stderr.write("\n".join(noise) + "\n")


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile all sources and link libtabnet.so (and the test library) next to this
    file; returns the product library's path."""
    srcs = SOURCES + TEST_SOURCES
    with tempfile.TemporaryDirectory(prefix="tabnet_build_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in srcs]
        with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            list(ex.map(_compile, srcs, objs))
        _link(objs[:len(SOURCES)], LIB)
        _link(objs, TEST_LIB)
    if verbose:
        print(f"built {LIB} and {TEST_LIB}")
    return LIB


def build_variant(defines, out: str) -> str:
    """Link a product library at `out` whose kernel source is compiled with the given
    preprocessor definitions (the tile sweep's candidate builds, which carry no generic
    entries); the other sources are compiled as for libtabnet.so."""
    srcs = [s for s in SOURCES if not s.startswith("tabnet_generic_")]
    with tempfile.TemporaryDirectory(prefix="tabnet_variant_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in srcs]
        with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            list(ex.map(lambda so: _compile(so[0], so[1], defines if so[0] == "tabnet_kernel.hip" else ()),
                        zip(srcs, objs)))
        _link(objs, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
