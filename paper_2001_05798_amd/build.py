"""Build libgwamg.so (HIP, gfx950) in-tree with hipcc.

Usage: python paper_2001_05798_amd/build.py  (or build() from Python).
Setup and assembly sources are compiled with -ffp-contract=off so that the
hierarchy is bit-reproducible; the solve sources may fuse multiply-adds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgwamg.so")
ARCH = os.environ.get("GWAMG_ARCH", "gfx950")

SOURCES = [
    ("runtime.cpp", False),
    ("util.hip", False),
    ("assemble.hip", True),
    ("setup.hip", True),
    ("sell.hip", False),
    ("solve.hip", False),
    ("noalloc.hip", False),
    ("batch.hip", False),
    ("sweep.hip", True),
    ("transient.hip", True),
    ("ilu.hip", True),
    ("capi.cpp", False),
    ("serve.cpp", False),
]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-result",
          f"-I{INCLUDE}", f"-I{CSRC}"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def _compile(src: str, exact: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc()] + COMMON + (["-ffp-contract=off"] if exact else ["-ffp-contract=fast"])
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda a: _compile(*a), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
