"""Build libfnscc.so (gfx950) in-tree with hipcc.

Usage: python -m paper_2506_06805_amd.build   (or __graft_entry__.build()).
Objects go to _build/ at the repository root; the library lands next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import shutil
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = ROOT / "_build"
LIB = PKG / "libfnscc.so"

SOURCES = [
    "fc_gemm.hip",
    "fc_split.hip",
    "fc_tensor.hip",
    "fc_integrals.hip",
    "fc_ccsd.hip",
    "fc_ladder.hip",
    "fc_sigma.hip",
    "fc_eom.hip",
    "fc_mlp.hip",
    "fc_aocd.hip",
    "fc_api.hip",
    "fc_linalg.cpp",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result", "-Wno-unused-function",
          f"-I{ROOT / 'include'}"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


# Host FP64 linear algebra on small complex matrices: plain complex products and quotients (no
# Annex G inf/nan recovery, which turns every complex multiply into a library call); the
# matrices are well scaled, far from overflow.
EXTRA = {"fc_linalg.cpp": ["-fcx-limited-range"]}


def _compile(src: str) -> pathlib.Path:
    s = CSRC / src
    obj = BUILD / (s.stem + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA.get(src, [])]
    cmd += ["-x", "hip", *DEVICE]
    cmd += ["-c", str(s), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> pathlib.Path:
    BUILD.mkdir(exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(str(tmp), str(LIB))
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
