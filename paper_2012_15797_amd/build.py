"""Builds libgfc.so (the HIP library behind include/gfc.h) for gfx950, in-tree.

    python -m paper_2012_15797_amd.build        # or build_library() from Python

Every HIP translation unit is compiled with hipcc for gfx950 only, with
packed-FP32 instruction selection disabled, and linked into one shared
library next to this file.
"""

from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_NAME = "libgfc.so"
LIB_PATH = os.path.join(PKG_DIR, LIB_NAME)
# rate probes for the roofline denominators (include/gfc_microbench.h)
MB_LIB_PATH = os.path.join(PKG_DIR, "libgfc_microbench.so")
MB_SOURCES = ["microbench.hip"]
ARCH = "gfx950"

SOURCES = [
    "gfc_error.cpp",
    "gfc_host.cpp",
    "sched.cpp",
    "render_dispatch.cpp",
    "render_fwd.hip",
    "render_w256.hip",
    "render_bwd.hip",
    "render_bwd_large.hip",
    "lanczos.hip",
    "sersic.hip",
    "psf_fft.hip",
    "serve.cpp",
]

HIPCC_FLAGS = [
    "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the gfx950 library cannot be built")


def _compile(src: str, obj: str) -> None:
    cmd = [_hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")


def _link(objs, path, libs=()):
    tmp = path + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *libs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, path)


def build_library(verbose: bool = False, jobs: int = 8) -> str:
    """Generates the twiddle table, compiles every source and links libgfc.so
    and the rate-probe library libgfc_microbench.so.  Always rebuilds.
    Returns the path of libgfc.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_twiddles.py"),
                    os.path.join(CSRC, "twiddles.inc")], check=True)
    srcs = [s for s in SOURCES + MB_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = {s: os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o") for s in srcs}
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, os.path.join(CSRC, s), o) for s, o in objs.items()]
        for f in futs:
            f.result()
    # roctx ranges of the host side (rocprofiler-sdk's roctx library)
    _link([objs[s] for s in SOURCES], LIB_PATH, ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                                                 "-Wl,-rpath,/opt/rocm/lib"])
    _link([objs[s] for s in MB_SOURCES], MB_LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH} from {len(SOURCES)} sources and {MB_LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build_library(verbose=True)
