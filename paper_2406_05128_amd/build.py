"""Build the gfx950 HIP library libtvlp.so in place (hipcc cross-compiles without a GPU).

The per-order launch sequences (tvlp_ops.hip) are compiled once per filter
order, each in its own process, next to the host API and the server and
synthesiser units; the objects are then linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtvlp.so")
OBJDIR = os.path.join(PKG, "_build")

SOURCES = ["tvlp_api.hip", "tvlp_serve.hip", "tvlp_sf.hip"]
ORDER_SOURCE = "tvlp_ops.hip"

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]

_NOISE = "is not a recognized feature for this target"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def compiled_orders() -> list[int]:
    """The orders the host API dispatches to (kOrders in tvlp_api.hip)."""
    with open(os.path.join(CSRC, "tvlp_api.hip")) as f:
        m = re.search(r"constexpr int kOrders\[\] = \{([^}]*)\}", f.read())
    return [int(x) for x in m.group(1).split(",")]


def _run(cmd: list[str]) -> str:
    proc = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in proc.stderr.splitlines() if _NOISE not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\nfailed ({proc.returncode}):\n{err}")
    return err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP unit (the order unit once per order) and link libtvlp.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = [f"-I{INCLUDE}", f"-I{CSRC}"]
    units = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        units.append([hipcc(), *HIPCC_FLAGS, *inc, "-c", "-o", obj, os.path.join(CSRC, src)])
    for m in compiled_orders():
        obj = os.path.join(OBJDIR, f"tvlp_ops_m{m}.o")
        units.append([hipcc(), *HIPCC_FLAGS, *inc, f"-DTVLP_ORDER={m}", "-c", "-o", obj,
                      os.path.join(CSRC, ORDER_SOURCE)])
    jobs = jobs or max(1, min(len(units), os.cpu_count() or 1, 16))
    if verbose:
        print(f"compiling {len(units)} units with {jobs} jobs", file=sys.stderr)
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for err in pool.map(_run, units):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    objs = [u[u.index("-o") + 1] for u in units]
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    shutil.rmtree(OBJDIR, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
