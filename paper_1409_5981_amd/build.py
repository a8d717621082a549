"""Build the HIP library libpmmm.so for gfx950 in-tree.

Every translation unit under csrc/ is compiled with hipcc for
--offload-arch=gfx950 (packed FP32 instructions disabled) and linked into
paper_1409_5981_amd/libpmmm.so, which the ctypes binding loads.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpmmm.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _newest_header() -> float:
    hdrs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max(os.path.getmtime(h) for h in hdrs)


# The column-stage unit is compiled once per (order, precision) and the
# hierarchy's fine-level unit once per order: the orders are the slowest part
# of the build, and apart they compile in parallel.
COLUMN_UNIT = "pmmm_column_inst.hip"
HIER_UNIT = "pmmm_hier_inst.hip"
PMAX = 10


def _units() -> list[tuple[str, str, list[str]]]:
    """(source, object name, extra flags) of every compile job, longest first."""
    units = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        base = os.path.basename(src).replace(".hip", "")
        if os.path.basename(src) == COLUMN_UNIT:
            for p in range(PMAX, -1, -1):
                for t in ("float", "double"):
                    units.append((src, f"{base}_p{p}_{t}",
                                  [f"-DPMMM_COLUMN_ORDER={p}", f"-DPMMM_COLUMN_T={t}"]))
        elif os.path.basename(src) == HIER_UNIT:
            for p in range(PMAX, -1, -1):
                units.append((src, f"{base}_p{p}", [f"-DPMMM_HIER_ORDER={p}"]))
        else:
            units.append((src, base, []))

    # high orders first, then the largest other units
    def order(u):
        return int(u[1].split("_p")[-1].split("_")[0])
    units.sort(key=lambda u: (-order(u) - 100 if u[0].endswith((COLUMN_UNIT, HIER_UNIT))
                              else -os.path.getsize(u[0]) / 1e6))
    return units


def _compile(unit: tuple[str, str, list[str]], incremental: bool = False) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(
            os.path.getmtime(src), _newest_header()):
        return obj
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every unit (incremental: only units older than their source or
    any header) and link libpmmm.so."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, incremental), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
