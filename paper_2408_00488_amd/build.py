"""Build the gfx950 shared library libcsl.so in-tree with hipcc.

Each HIP source is compiled to an object in its own hipcc process (in
parallel), then the objects are linked into libcsl.so.

Usage: python -m paper_2408_00488_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcsl.so")
SOURCES = ["csl_kernels.hip", "csl_kernels_wg256h.hip", "csl_kernels_wg512.hip",
           "csl_kernels_wg512x.hip", "csl_kernels_wg1024p.hip", "csl_kernels_wg512p.hip",
           "csl_runtime.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every HIP source for gfx950 into libcsl.so (always rebuilds)."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="csl_build_") as tmpdir:
        procs, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [cc] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
                                  "-o", obj] + (extra or [])
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = []
        for src, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                sys.stderr.write(out)
                failed.append(src)
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        tmp = LIB + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-fPIC", "-shared"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
