"""Build step for the HIP library (``libiqa_hip.so``, gfx950 only).

Run as ``python -m paper_2501_10653_amd.build``; ``__graft_entry__.build()``
calls :func:`build` too.  The library is built in-tree, next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = [os.path.join(PKG, "csrc", "iqa_kernels.hip")]
LIB = os.path.join(PKG, "libiqa_hip.so")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# -ffp-contract=off: every multiply-add the kernels want is an explicit fmaf,
#   so compensated sums and the double-float finalisation round as written.
# -packed-fp32-ops off: no v_pk_* FP32 instructions are generated.
HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into ``libiqa_hip.so`` (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *HIPFLAGS, *SOURCES, "-o", tmp]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 target feature: harmless
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
