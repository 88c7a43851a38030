"""Shared helpers for the GPU parity tests: run the HIP path, run the oracle on
the same inputs, and compare with the tolerance rule of the precision contract.

Tolerance (per tile, FP32 kernel vs FP64 oracle):
  * LISI and the sums A, P, Sx, Sy are ratios / sums of non-negative terms, so
    plain relative error is well posed: |g - o| <= 1e-5 * |o| (0 vs 0 passes).
  * augLISI = 1 - r with r = P/(Sx+Sy+C) loses relative accuracy as r -> 1;
    it passes when |g - o| <= 1e-5 * max(|o|, r_o), i.e. plain relative error
    whenever augLISI >= 0.5, and error relative to r below that.
"""

from __future__ import annotations

from typing import Optional

import numpy as np
import pytest
import torch

from oracle import oracle

TOL = 1e-5
C6 = 1e-6

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP GPU")


def dev():
    return torch.device("cuda", 0)


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev())


def oracle_for(x, y, NT, C1=C6, C2=C6, C=C6, D=None):
    """Oracle at the float32 values of the constants the kernel receives."""
    C1f, C2f, Cf = (oracle.f32const(v) for v in (C1, C2, C))
    Df = oracle.f32const(D) if D is not None else C1f / 2.0
    return oracle.iqa_tiles(x, y, NT, Df, C1f, C2f, Cf)


def rel_errors(g: np.ndarray, o: np.ndarray) -> np.ndarray:
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    den = np.abs(o)
    err = np.abs(g - o)
    return np.where(den > 0, err / np.where(den > 0, den, 1.0), np.where(err > 0, np.inf, 0.0))


def aug_errors(g: np.ndarray, o: np.ndarray) -> np.ndarray:
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = np.maximum(np.abs(o), np.abs(1.0 - o))
    return np.abs(g - o) / scale


def assert_parity(res, ora, tol: float = TOL, what: str = "",
                  sample: Optional[np.ndarray] = None) -> dict:
    """Compare a TileResult against oracle output; returns error statistics."""
    ol, oa, osum = ora
    stats = {}
    if res.lisi is not None:
        g = res.lisi.cpu().numpy().ravel()
        e = rel_errors(g, ol.ravel())
        stats["lisi_max_rel"] = float(e.max())
        assert e.max() <= tol, f"{what} LISI max rel err {e.max():.3g} at tile {int(e.argmax())}"
    if res.auglisi is not None:
        g = res.auglisi.cpu().numpy().ravel()
        e = aug_errors(g, oa.ravel())
        stats["aug_max_err"] = float(e.max())
        stats["aug_max_plain_rel"] = float(rel_errors(g, oa.ravel()).max())
        assert e.max() <= tol, f"{what} augLISI err {e.max():.3g} at tile {int(e.argmax())}"
    if res.sums is not None:
        g = res.sums.cpu().numpy()
        for k, name in enumerate("A P Sx Sy".split()):
            e = rel_errors(g[:, k], osum[:, k])
            stats[f"{name}_max_rel"] = float(e.max())
            assert e.max() <= tol, f"{what} sum {name} max rel err {e.max():.3g}"
    return stats
