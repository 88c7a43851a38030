"""ctypes front end of the FP64 CPU oracle (``oracle/iqa_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It computes
Eq. (1) and Eq. (2) of the paper tile by tile in double precision after the
negative-pixel clamp of Section 2, and merges tiles with Eq. (3) and Eq. (4).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "iqa_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Plain optimisation, no fast-math and no contraction into fused multiply-adds,
# so every operation rounds exactly as written.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Werror"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib: Optional[ctypes.CDLL] = None


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = os.environ.get("IQA_ORACLE_LIB")   # mutation tests load a planted copy
        if not path:
            if not os.path.exists(LIB):
                build()
            path = LIB
        lib = ctypes.CDLL(path)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        d = ctypes.c_double
        lib.oracle_iqa_tiles.argtypes = [f32p, f32p, i64, i64, d, d, d, d, f64p, f64p, f64p]
        lib.oracle_iqa_tiles.restype = ctypes.c_int
        lib.oracle_merge_tiles.argtypes = [f64p, f64p, f64p, i64, i64, d, d, f64p, f64p, f64p]
        lib.oracle_merge_tiles.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _f32(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def f32const(v: float) -> float:
    """The double value of a constant after rounding to float32, i.e. exactly
    what an FP32 kernel sees when handed the same constant."""
    return float(np.float32(v))


def iqa_tiles(x: np.ndarray, y: np.ndarray, NT: int, D: float, C1: float,
              C2: float, C: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Per-tile LISI, augLISI (each (N/NT, N/NT) float64) and sums (n, 4):
    A, P, Sx, Sy.  Constants are used exactly as given (pass ``f32const``
    values to mirror an FP32 kernel)."""
    x = _f32(x)
    y = _f32(y)
    if x.ndim != 2 or x.shape[0] != x.shape[1] or x.shape != y.shape:
        raise ValueError(f"expected two equal N x N images, got {x.shape} and {y.shape}")
    N = x.shape[0]
    if NT <= 0 or N % NT:
        raise ValueError(f"N={N} is not a positive multiple of NT={NT}")
    ns = N // NT
    lisi = np.empty((ns, ns), np.float64)
    aug = np.empty((ns, ns), np.float64)
    sums = np.empty((ns * ns, 4), np.float64)
    rc = _load().oracle_iqa_tiles(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float), N, NT,
                                  D, C1, C2, C, _ptr(lisi, ctypes.c_double),
                                  _ptr(aug, ctypes.c_double), _ptr(sums, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"oracle_iqa_tiles failed with status {rc}")
    return lisi, aug, sums


def merge_tiles(lisi: np.ndarray, aug: np.ndarray, sums: np.ndarray, f: int,
                C2: float, C: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Eq. (3)/(4): merge f x f blocks of tiles into parent tiles."""
    lisi = np.ascontiguousarray(lisi, np.float64)
    aug = np.ascontiguousarray(aug, np.float64)
    sums = np.ascontiguousarray(sums, np.float64).reshape(-1, 4)
    ns = lisi.shape[0]
    if f <= 0 or ns % f:
        raise ValueError(f"{ns} tiles per side is not a multiple of {f}")
    npar = ns // f
    lp = np.empty((npar, npar), np.float64)
    ap = np.empty((npar, npar), np.float64)
    sp = np.empty((npar * npar, 4), np.float64)
    rc = _load().oracle_merge_tiles(_ptr(lisi, ctypes.c_double), _ptr(aug, ctypes.c_double),
                                    _ptr(sums, ctypes.c_double), ns, f, C2, C,
                                    _ptr(lp, ctypes.c_double), _ptr(ap, ctypes.c_double),
                                    _ptr(sp, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"oracle_merge_tiles failed with status {rc}")
    return lp, ap, sp


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for later calls (results are bitwise the same)."""
    _load().oracle_set_num_threads(int(n))
