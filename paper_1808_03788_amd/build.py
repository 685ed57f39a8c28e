"""Build libader.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1808_03788_amd.build          # compile every unit, link

Every HIP unit is compiled with -Xclang -target-feature -Xclang -packed-fp32-ops
(no packed FP32 instructions); objects go to _build/ at the repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libader.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("ADER_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, object name, extra flags): the kernel instantiations are compiled
# once per (family, degree) so that they build in parallel
FAMILIES = [("euler2", 2, 0), ("euler3", 3, 0), ("elastic3", 3, 1)]
UNITS = [("api.hip", "api", []), ("basis.cpp", "basis", [])] + [
    ("inst_degree.hip", f"inst_{fam}_N{N}", [f"-DADER_DIM={dim}", f"-DADER_ELASTIC={el}", f"-DADER_DEGREE={N}"])
    for fam, dim, el in FAMILIES for N in range(8)]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(unit) -> str:
    name, tag, extra = unit
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, tag + ".o")
    lang = ["-x", "hip"] if name.endswith(".hip") else []
    cmd = [HIPCC, *FLAGS, *extra, *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {tag}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
