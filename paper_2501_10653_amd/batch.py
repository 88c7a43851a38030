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
from .iqa import C_DEFAULT, TileResult, _check_images, _mark_used, _stream_handle, default_D


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
    N x N device tensors.  Pairs with NT % 4 == 0 and 16-byte aligned images go
    into the persistent launch; any others are launched one by one on the same
    stream.  Output tensors are allocated here and reused by every run:
    ``results[i]`` is the :class:`TileResult` of pair i.
    """

    def __init__(self, pairs: Sequence, *, C1: float = C_DEFAULT, C2: float = C_DEFAULT,
                 C: float = C_DEFAULT, D: Optional[float] = None, sums: bool = False,
                 waves: Optional[int] = None, device: Optional[torch.device] = None,
                 inline: Optional[bool] = None):
        if len(pairs) == 0:
            raise ValueError("empty batch")
        if D is None:
            D = default_D(C1)
        self.consts = dict(C1=C1, C2=C2, C=C, D=D)
        self.device = device or pairs[0][0].device
        self.waves = int(waves) if waves is not None else default_waves()
        self.inputs = []
        self.results: List[TileResult] = []
        self.bytes = 0
        batched, self.single = [], []      # pairs the persistent kernel takes / does not
        # Every output is a view into one buffer (each array at a 16-byte
        # aligned offset): one allocation, and one stream record per run.
        sizes = []
        for x, y, NT in pairs:
            N = _check_images(x, y)
            ns = N // NT if NT > 0 and N % NT == 0 else 0
            sizes.append(ns)
        pad = lambda n: (n + 3) // 4 * 4
        per = [2 * pad(ns * ns) + (pad(4 * ns * ns) if sums else 0) for ns in sizes]
        self.out = torch.empty(max(1, sum(per)), device=self.device)
        off = 0
        for i, ((x, y, NT), ns) in enumerate(zip(pairs, sizes)):
            N = x.shape[0]
            lo = self.out[off:off + ns * ns].view(ns, ns)
            off += pad(ns * ns)
            ao = self.out[off:off + ns * ns].view(ns, ns)
            off += pad(ns * ns)
            so = None
            if sums:
                so = self.out[off:off + 4 * ns * ns].view(ns * ns, 4)
                off += pad(4 * ns * ns)
            self.inputs.append((x, y, NT))
            self.results.append(TileResult(lo, ao, so))
            self.bytes += 8 * N * N
            vec4 = NT % 4 == 0 and x.data_ptr() % 16 == 0 and y.data_ptr() % 16 == 0
            (batched if vec4 else self.single).append(i)
        self.count = len(batched)
        self.units = 0
        self.descs = None
        self.descs_host = None
        # Up to BATCH_INLINE_MAX pairs travel in the kernel arguments (no
        # device table); `inline` forces either form.
        self.inline = (self.count <= _lib.BATCH_INLINE_MAX) if inline is None else bool(inline)
        if self.inline and self.count > _lib.BATCH_INLINE_MAX:
            raise ValueError(f"inline batches hold at most {_lib.BATCH_INLINE_MAX} pairs")
        if batched:
            arr = (IqaPair * len(batched))()
            for k, i in enumerate(batched):
                x, y, NT = self.inputs[i]
                r = self.results[i]
                arr[k] = IqaPair(x.data_ptr(), y.data_ptr(), x.shape[0], NT, D, C1, C2, C,
                                 r.lisi.data_ptr(), r.auglisi.data_ptr(),
                                 r.sums.data_ptr() if r.sums is not None else None)
            host = np.zeros(len(batched) * _lib.BATCH_DESC_BYTES, np.uint8)
            units = ctypes.c_int64(0)
            _lib.check(_lib.load().iqa_batch_describe(arr, len(batched), host.ctypes.data,
                                                      ctypes.byref(units)), "iqa_batch_describe")
            self.units = int(units.value)
            if self.inline:
                self.descs_host = host
            else:
                self.descs = torch.from_numpy(host).to(self.device)   # device copy, 256-B aligned

    def run(self, stream=None) -> None:
        """Enqueue the batch: one persistent launch over every pair with
        N_T % 4 == 0 and 16-byte aligned images (descriptors in the kernel
        arguments or in a device table), and a single-pair launch for each of
        the others, all on the same stream."""
        from .iqa import iqa_tiles
        with torch.cuda.device(self.device):
            if self.descs_host is not None:
                st = _lib.load().iqa_tiles_batched_inline(self.descs_host.ctypes.data, self.count,
                                                          self.units, self.waves,
                                                          _stream_handle(self.device, stream))
                _lib.check(st, "iqa_tiles_batched_inline")
            elif self.descs is not None:
                st = _lib.load().iqa_tiles_batched(self.descs.data_ptr(), self.count, self.units,
                                                   self.waves,
                                                   _stream_handle(self.device, stream))
                _lib.check(st, "iqa_tiles_batched")
            for i in self.single:
                x, y, NT = self.inputs[i]
                r = self.results[i]
                out = {"lisi": r.lisi, "auglisi": r.auglisi}
                if r.sums is not None:
                    out["sums"] = r.sums
                iqa_tiles(x, y, NT, sums=r.sums is not None, out=out, stream=stream,
                          **self.consts)
            # the outputs and the descriptor table were allocated on torch's
            # current stream; the launches may run on another torch stream
            _mark_used(stream, self.descs, self.out)

    def capture(self, stream: Optional[torch.cuda.Stream] = None) -> torch.cuda.CUDAGraph:
        """Capture one run into a HIP graph; replay it with ``graph.replay()``
        under ``torch.cuda.stream(stream)``."""
        stream = stream or torch.cuda.Stream(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            self.run(stream=stream)
        return g
