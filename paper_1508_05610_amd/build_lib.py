"""Build liblf2.so (HIP, gfx950) in-tree.

Each translation unit is compiled to an object file under ``_build/`` in
parallel, then linked into ``paper_1508_05610_amd/liblf2.so``.  Always
recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblf2.so")
ARCH = os.environ.get("LF2_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]

# (source, extra flags, object name)
UNITS = [
    ("lf2_kx.hip", ["-DLF2_KX_PART=0"], "kx_r2c.o"),
    ("lf2_kx.hip", ["-DLF2_KX_PART=1"], "kx_c2r.o"),
    ("lf2_kx.hip", ["-DLF2_KX_PART=2"], "kx_c2c.o"),
    ("lf2_ks.hip", [], "ks.o"),
    ("lf2_kreg.hip", [], "kreg.o"),
    ("lf2_kmisc.hip", [], "kmisc.o"),
    ("lf2_kbatch.hip", [], "kbatch.o"),
    ("lf2_kgen.hip", [], "kgen.o"),
    ("lf2_api.cpp", ["-x", "hip"], "api.o"),
    ("lf2_batch.cpp", ["-x", "hip"], "batch.o"),
    ("lf2_server.cpp", ["-x", "hip"], "server.o"),
    ("lf2_kfield.hip", [], "kfield.o"),
    ("lf2_field.cpp", ["-x", "hip"], "field.o"),
]


def _compile(unit):
    src, extra, obj = unit
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out, r.stderr


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, UNITS))
    objs = [o for o, _ in results]
    if verbose:
        for o, err in results:
            if err.strip():
                print(f"[{os.path.basename(o)}]\n{err}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
