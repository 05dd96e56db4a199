"""Build libmatgraph.so (HIP for gfx950) in-tree, next to this file.

    python -m paper_2307_05380_amd.build [--verbose]

Every translation unit under ``csrc/`` is compiled with hipcc for gfx950 only,
then linked into one shared library with the C ABI of ``include/matgraph.h``.
Packed FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmatgraph.so")
SOURCES = ["api.hip", "bounds.hip", "sweep.hip", "knn.hip", "celllist.hip", "geometry.hip", "triplets.hip", "symmetrize.hip", "ties.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    out = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in line and "not a recognized feature" not in line
                    and line.strip() != "1 warning generated." and line.strip())
    if verbose and out:
        print(out, flush=True)
    return r


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source for gfx950 and link libmatgraph.so. Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    flags = compile_flags()
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 4)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    path = build(verbose="--verbose" in argv or "-v" in argv)
    print(path)


if __name__ == "__main__":
    main()
