"""Builds the HIP library libads.so for gfx950 in-tree (paper_2303_09855_amd/_lib).

Every translation unit is compiled to an object in parallel, then linked.  The
scan kernel's template instantiations are split into one object per (storage
type, block width) by compiling scan_inst.hip with different macro values.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIB = os.path.join(LIBDIR, "libads.so")
SOURCES = ["api.hip", "scan.hip", "gemm.hip", "dco.hip", "kmeans.hip", "hnsw.hip"]
SCAN_DTYPES = [0, 1, 2]          # ADS_F32, ADS_BF16, ADS_F16
SCAN_WIDTHS = [8, 16, 32, 64]    # supported block widths of the stored layout

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep packed FP32 instructions out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _units():
    """(source, object, extra flags) of every translation unit."""
    out = [(s, s.replace(".hip", ".o"), []) for s in SOURCES]
    for dt in SCAN_DTYPES:
        for dd in SCAN_WIDTHS:
            out.append(("scan_inst.hip", f"scan_inst_{dt}_{dd}.o",
                        [f"-DADS_SCAN_DT={dt}", f"-DADS_SCAN_DD={dd}"]))
    return out


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed: {' '.join(cmd)}")
    noisy = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noisy and verbose:
        sys.stderr.write("\n".join(noisy) + "\n")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit (always recompiles) and link libads.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(HERE, os.pardir, "include")]
    units = _units()
    cmds = [[hipcc(), *HIPCC_FLAGS, *inc, *extra, "-c", os.path.join(CSRC, src),
             "-o", os.path.join(OBJDIR, obj)] for src, obj, extra in units]
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
          *[os.path.join(OBJDIR, obj) for _, obj, _ in units], "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
