"""Ragged batches: many image pairs of mixed N and N_T in one persistent launch.

:class:`Batch` plans a batch once (host-side descriptors from the C library,
copied to the device), then :meth:`Batch.run` issues one launch of the
persistent kernel.  The launch allocates nothing, so a run can be captured
into a HIP graph (:meth:`Batch.capture`) and replayed.  Argument marshalling
only; every step of the computation runs in ``libiqa_hip.so``.
"""

from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import IqaPair, LaunchCfg
from .iqa import C_DEFAULT, TileResult, _check_images, _stream_handle, default_D


def default_waves() -> int:
    """Persistent waves per batch launch: the autotuned value compiled into the
    library (8 per CU on 256 CUs when untuned)."""
    return int(_lib.load().iqa_batch_default_waves())


def batch_cfg(N: int, NT: int) -> dict:
    """Per-pair geometry a batch uses for (N, NT) (results bitwise equal to
    ``iqa_tiles(..., cfg=batch_cfg(N, NT))``)."""
    c = LaunchCfg()
    _lib.check(_lib.load().iqa_batch_cfg(N, NT, ctypes.byref(c)), "iqa_batch_cfg")
    return c.as_dict()


class Batch:
    """A planned ragged batch.

    ``pairs`` is a sequence of ``(x, y, NT)`` with x, y contiguous float32
    N x N device tensors (16-byte aligned, NT % 4 == 0).  Output tensors are
    allocated here and reused by every run: ``results[i]`` is the
    :class:`TileResult` of pair i.
    """

    def __init__(self, pairs: Sequence, *, C1: float = C_DEFAULT, C2: float = C_DEFAULT,
                 C: float = C_DEFAULT, D: Optional[float] = None, sums: bool = False,
                 waves: Optional[int] = None, device: Optional[torch.device] = None):
        if len(pairs) == 0:
            raise ValueError("empty batch")
        if D is None:
            D = default_D(C1)
        self.device = device or pairs[0][0].device
        self.waves = int(waves) if waves is not None else default_waves()
        self.inputs = []
        self.results: List[TileResult] = []
        arr = (IqaPair * len(pairs))()
        self.bytes = 0
        for i, (x, y, NT) in enumerate(pairs):
            N = _check_images(x, y)
            ns = N // NT if NT > 0 and N % NT == 0 else 0
            lo = torch.empty(ns, ns, device=self.device)
            ao = torch.empty(ns, ns, device=self.device)
            so = torch.empty(ns * ns, 4, device=self.device) if sums else None
            self.inputs.append((x, y, NT))
            self.results.append(TileResult(lo, ao, so))
            arr[i] = IqaPair(x.data_ptr(), y.data_ptr(), N, NT, D, C1, C2, C, lo.data_ptr(),
                             ao.data_ptr(), so.data_ptr() if so is not None else None)
            self.bytes += 8 * N * N
        host = np.zeros(len(pairs) * _lib.BATCH_DESC_BYTES, np.uint8)
        units = ctypes.c_int64(0)
        _lib.check(_lib.load().iqa_batch_describe(arr, len(pairs), host.ctypes.data,
                                                  ctypes.byref(units)), "iqa_batch_describe")
        self.count = len(pairs)
        self.units = int(units.value)
        self.descs = torch.from_numpy(host).to(self.device)   # device copy, 256-B aligned

    def run(self, stream=None) -> None:
        """Enqueue one persistent launch over the whole batch."""
        with torch.cuda.device(self.device):
            st = _lib.load().iqa_tiles_batched(self.descs.data_ptr(), self.count, self.units,
                                               self.waves, _stream_handle(self.device, stream))
        _lib.check(st, "iqa_tiles_batched")

    def capture(self, stream: Optional[torch.cuda.Stream] = None) -> torch.cuda.CUDAGraph:
        """Capture one run into a HIP graph; replay it with ``graph.replay()``
        under ``torch.cuda.stream(stream)``."""
        stream = stream or torch.cuda.Stream(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            self.run(stream=stream)
        return g
