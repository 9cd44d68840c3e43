"""Build libgce.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgce.so")
# command-line search over inputs in raw files, linked against libgce.so only
FILE_SEARCH = os.path.join(PKG, "gce_file_search")
# the search-kernel variants are spread over four files so they compile in
# parallel
SOURCES = ["gce_kernels.hip", "gce_search_fp64.hip", "gce_search_fp64_overlap.hip",
           "gce_search_split.hip", "gce_search_split_overlap.hip", "gce_noalloc.hip",
           "gce_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: the only fused multiply-adds are the explicit ones, so
# the FP64 fold reproduces the documented operation sequence bit for bit.
# Packed FP32 VALU ops are disabled for the device code.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; drop that note
    noise = "'-packed-fp32-ops' is not a recognized feature"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel) and link libgce.so next to this
    file; returns its path."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="gce_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC, *FLAGS, "-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
        os.replace(tmp, LIB)
        ftmp = FILE_SEARCH + ".tmp%d" % os.getpid()
        _run([HIPCC, "-O2", "-std=c++17", "-Wall", "-I", INCLUDE,
              os.path.join(CSRC, "gce_file_search.cpp"), "-L", PKG, "-lgce",
              "-Wl,-rpath,$ORIGIN", "-o", ftmp], verbose)
    os.replace(ftmp, FILE_SEARCH)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
