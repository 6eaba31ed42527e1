"""Builds libpic.so (the HIP library behind include/pic.h) for gfx950 with hipcc.

Usage:  python -m paper_2106_12919_amd.build   (or build() from Python).
Each translation unit is compiled to an object in ``_build/`` in parallel, then
linked in-tree to ``paper_2106_12919_amd/libpic.so``.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpic.so")
SOURCES = ["api.hip", "fft.hip", "centering.hip", "psatd.hip", "particles.hip", "sort.hip", "diag.hip", "tables.cpp",
           "probe.hip"]

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found (ROCm is required to build libpic)")
    return h


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS + list(extra)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return src, obj, r.returncode, r.stdout


def build(verbose=False, jobs=None, out=LIB, build_dir=BUILD, extra_flags=()):
    """Compile every source and link ``out`` (default: the in-tree libpic.so).

    ``extra_flags`` (e.g. -D tuning macros) and another ``out``/``build_dir`` build a variant
    for A/B timing without touching the in-tree library.  Raises RuntimeError on failure."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, build_dir, extra_flags), SOURCES))
    errors = [(s, log) for s, _, rc, log in results if rc != 0]
    for s, _, rc, log in results:
        if verbose and log.strip():
            print(f"--- {s}\n{log}")
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(f"--- {s}\n{log}" for s, log in errors))
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-o", tmp] + [o for _, o, _, _ in results] + [f"--offload-arch={ARCH}", "-fPIC"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
