"""Python binding of the tile-wise LISI / augLISI library.

Argument marshalling only: tensors are checked, outputs are allocated with
torch on the inputs' device, and the C entry points of ``libiqa_hip.so`` do
all of the work on the caller's (or torch's current) HIP stream.  The names
mirror the C ABI: :func:`iqa_tiles`, :func:`lisi_tiles`, :func:`auglisi_tiles`.
"""

from __future__ import annotations

import ctypes
from typing import Dict, NamedTuple, Optional

import torch

from . import _lib
from ._lib import IqaError, LaunchCfg

# The paper only asks C1, C2, C << 1; these defaults are 1e-6 each and D is
# C1/2, the choice for which identical tiles give LISI = S/(S + C2) ~ 1.
C_DEFAULT = 1e-6


def default_D(C1: float) -> float:
    """D = C1/2, computed on the float32 value of C1."""
    import numpy as np
    return float(np.float32(C1)) / 2.0


class TileResult(NamedTuple):
    lisi: Optional[torch.Tensor]
    auglisi: Optional[torch.Tensor]
    sums: Optional[torch.Tensor]


def _check_images(x: torch.Tensor, y: torch.Tensor) -> int:
    for name, t in (("x", x), ("y", y)):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must live on a HIP device, got {t.device}")
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32, got {t.dtype}")
        if t.dim() != 2 or t.shape[0] != t.shape[1]:
            raise ValueError(f"{name} must be N x N, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous (row-major)")
    if x.shape != y.shape or x.device != y.device:
        raise ValueError("x and y must have the same shape and device")
    return int(x.shape[0])


def _stream_handle(device: torch.device, stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _mark_used(stream, *tensors) -> None:
    """Outputs allocated here on torch's current stream but written on another
    torch stream: tell the caching allocator, so that their memory is not
    handed out again before that stream has finished with it.  Under graph
    capture nothing runs yet; the captured launches use the memory whenever
    the graph is replayed, so the caller keeps those tensors alive."""
    if isinstance(stream, torch.cuda.Stream) and not torch.cuda.is_current_stream_capturing():
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def _out(shape, device, given: Optional[torch.Tensor], name: str) -> torch.Tensor:
    if given is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    if tuple(given.shape) != tuple(shape) or given.dtype != torch.float32 or \
            not given.is_contiguous() or given.device != device:
        raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape} on {device}")
    return given


def iqa_tiles(x: torch.Tensor, y: torch.Tensor, NT: int, *, C1: float = C_DEFAULT,
              C2: float = C_DEFAULT, C: float = C_DEFAULT, D: Optional[float] = None,
              lisi: bool = True, auglisi: bool = True, sums: bool = False,
              cfg: Optional[dict] = None, stream=None,
              out: Optional[Dict[str, torch.Tensor]] = None) -> TileResult:
    """Fused per-tile LISI (Eq. 1) and augLISI (Eq. 2) of two N x N images.

    Returns (N/NT, N/NT) float32 matrices (row-major tiles) and, when asked,
    the (n, 4) per-tile sums A, P, Sx, Sy.  Work is enqueued on ``stream``
    (default: torch's current stream) and not waited for."""
    N = _check_images(x, y)
    if D is None:
        D = default_D(C1)
    out = out or {}
    ns = N // NT if NT > 0 and N % NT == 0 else 0
    dev = x.device
    lo = _out((ns, ns), dev, out.get("lisi"), "lisi") if lisi else None
    ao = _out((ns, ns), dev, out.get("auglisi"), "auglisi") if auglisi else None
    so = _out((ns * ns, 4), dev, out.get("sums"), "sums") if sums else None
    lib = _lib.load()
    cfg_p = ctypes.byref(LaunchCfg.from_dict(cfg)) if cfg is not None else None
    with torch.cuda.device(dev):
        st = lib.iqa_tiles_cfg(_ptr(x), _ptr(y), N, NT, D, C1, C2, C, _ptr(lo), _ptr(ao),
                               _ptr(so), cfg_p, _stream_handle(dev, stream))
    _lib.check(st, "iqa_tiles")
    _mark_used(stream, *(t for k, t in (("lisi", lo), ("auglisi", ao), ("sums", so))
                         if k not in out))
    return TileResult(lo, ao, so)


def lisi_tiles(x: torch.Tensor, y: torch.Tensor, NT: int, *, C1: float = C_DEFAULT,
               C2: float = C_DEFAULT, D: Optional[float] = None, stream=None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-tile LISI (Eq. 1) only; bitwise equal to iqa_tiles' LISI output."""
    N = _check_images(x, y)
    if D is None:
        D = default_D(C1)
    ns = N // NT if NT > 0 and N % NT == 0 else 0
    lo = _out((ns, ns), x.device, out, "out")
    with torch.cuda.device(x.device):
        st = _lib.load().lisi_tiles(_ptr(x), _ptr(y), N, NT, D, C1, C2, _ptr(lo),
                                    _stream_handle(x.device, stream))
    _lib.check(st, "lisi_tiles")
    if out is None:
        _mark_used(stream, lo)
    return lo


def auglisi_tiles(x: torch.Tensor, y: torch.Tensor, NT: int, *, C: float = C_DEFAULT,
                  stream=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Per-tile augLISI (Eq. 2) only; bitwise equal to iqa_tiles' output."""
    N = _check_images(x, y)
    ns = N // NT if NT > 0 and N % NT == 0 else 0
    ao = _out((ns, ns), x.device, out, "out")
    with torch.cuda.device(x.device):
        st = _lib.load().auglisi_tiles(_ptr(x), _ptr(y), N, NT, C, _ptr(ao),
                                       _stream_handle(x.device, stream))
    _lib.check(st, "auglisi_tiles")
    if out is None:
        _mark_used(stream, ao)
    return ao


def default_cfg(N: int, NT: int, x: Optional[torch.Tensor] = None,
                y: Optional[torch.Tensor] = None) -> dict:
    """The launch configuration iqa_tiles picks for (N, NT) (and the images'
    alignment; 256-byte aligned pointers are assumed when none are given)."""
    c = LaunchCfg()
    px = _ptr(x) if x is not None else 256
    py = _ptr(y) if y is not None else 256
    _lib.check(_lib.load().iqa_default_cfg(N, NT, px, py, ctypes.byref(c)), "iqa_default_cfg")
    return c.as_dict()


def check_cfg(N: int, NT: int, cfg: dict) -> int:
    """Status of an explicit configuration for (N, NT): 0 when valid."""
    return int(_lib.load().iqa_check_cfg(N, NT, ctypes.byref(LaunchCfg.from_dict(cfg))))


def prepare(N: int, NT: int, cfg: Optional[dict] = None, stream=None,
            device: Optional[torch.device] = None) -> None:
    """Allocate the split workspace (N, NT, cfg) needs on ``stream`` ahead of
    graph capture."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    cfg_p = ctypes.byref(LaunchCfg.from_dict(cfg)) if cfg is not None else None
    with torch.cuda.device(device):
        st = _lib.load().iqa_prepare(N, NT, cfg_p, _stream_handle(device, stream))
    _lib.check(st, "iqa_prepare")


def read_ceiling(buf: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    """Streaming-read reference kernel (measurement only): one float per
    workgroup into ``out``; the number of workgroups is ``out.numel()``."""
    if buf.dtype != torch.float32 or not buf.is_contiguous() or out.dtype != torch.float32:
        raise ValueError("read_ceiling needs contiguous float32 tensors")
    with torch.cuda.device(buf.device):
        st = _lib.load().iqa_read_ceiling(buf.data_ptr(), buf.numel(), out.data_ptr(),
                                          out.numel(), _stream_handle(buf.device, stream))
    _lib.check(st, "iqa_read_ceiling")


def launch_workgroups(N: int, NT: int, cfg: dict) -> int:
    """Workgroups of the single-pair launch for (N, NT) with ``cfg``."""
    n = int(_lib.load().iqa_launch_workgroups(N, NT, ctypes.byref(LaunchCfg.from_dict(cfg))))
    if n < 0:
        raise ValueError(f"invalid shape or configuration: {N} {NT} {cfg}")
    return n


def tiles_timeline(x: torch.Tensor, y: torch.Tensor, NT: int, cfg: dict, stamps: torch.Tensor,
                   *, C1: float = C_DEFAULT, C2: float = C_DEFAULT, C: float = C_DEFAULT,
                   D: Optional[float] = None, stream=None,
                   out: Optional[Dict[str, torch.Tensor]] = None) -> TileResult:
    """The fused launch with a per-workgroup timeline (diagnostics): ``stamps``
    is an int64 tensor of at least 8 entries per workgroup (see
    :func:`launch_workgroups`) that receives wall-clock stamps, hardware ids,
    tile group and split part of every workgroup."""
    N = _check_images(x, y)
    if D is None:
        D = default_D(C1)
    if stamps.dtype != torch.int64 or not stamps.is_contiguous() or stamps.device != x.device:
        raise ValueError("stamps must be a contiguous int64 tensor on the images' device")
    ns = N // NT if NT > 0 and N % NT == 0 else 0
    out = out or {}
    lo = _out((ns, ns), x.device, out.get("lisi"), "lisi")
    ao = _out((ns, ns), x.device, out.get("auglisi"), "auglisi")
    with torch.cuda.device(x.device):
        st = _lib.load().iqa_tiles_timeline(
            _ptr(x), _ptr(y), N, NT, D, C1, C2, C, _ptr(lo), _ptr(ao), None,
            ctypes.byref(LaunchCfg.from_dict(cfg)), stamps.data_ptr(), stamps.numel(),
            _stream_handle(x.device, stream))
    _lib.check(st, "iqa_tiles_timeline")
    return TileResult(lo, ao, None)


def probe_empty(blocks: int, threads: int, stream=None, device=None) -> None:
    """One launch of an empty kernel (measurement only)."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(device):
        st = _lib.load().iqa_probe_empty(blocks, threads, _stream_handle(device, stream))
    if st != _lib.IQA_OK:
        raise IqaError(st, "iqa_probe_empty", _lib.load().iqa_probe_last_hip_error())


def probe_read(buf: torch.Tensor, out: torch.Tensor, threads: int, loads: int, mode: int,
               stream=None) -> None:
    """A plain read of ``buf`` by ``out.numel()`` workgroups (measurement only)."""
    if buf.dtype != torch.float32 or not buf.is_contiguous() or out.dtype != torch.float32:
        raise ValueError("probe_read needs contiguous float32 tensors")
    with torch.cuda.device(buf.device):
        st = _lib.load().iqa_probe_read(buf.data_ptr(), buf.numel(), out.data_ptr(), out.numel(),
                                        threads, loads, mode, _stream_handle(buf.device, stream))
    if st != _lib.IQA_OK:
        raise IqaError(st, "iqa_probe_read", _lib.load().iqa_probe_last_hip_error())


def probe_read_timeline(buf: torch.Tensor, out: torch.Tensor, threads: int, loads: int,
                        stamps: torch.Tensor, stream=None) -> None:
    """The register read of ``buf`` by ``out.numel()`` workgroups with
    per-workgroup wall-clock stamps into ``stamps`` (int64, 8 per workgroup;
    the layout of :func:`tiles_timeline`).  Measurement only."""
    if buf.dtype != torch.float32 or not buf.is_contiguous() or out.dtype != torch.float32:
        raise ValueError("probe_read_timeline needs contiguous float32 tensors")
    if stamps.dtype != torch.int64 or not stamps.is_contiguous() or stamps.device != buf.device:
        raise ValueError("stamps must be a contiguous int64 tensor on the buffer's device")
    with torch.cuda.device(buf.device):
        st = _lib.load().iqa_probe_read_timeline(buf.data_ptr(), buf.numel(), out.data_ptr(),
                                                 out.numel(), threads, loads, stamps.data_ptr(),
                                                 stamps.numel(),
                                                 _stream_handle(buf.device, stream))
    if st != _lib.IQA_OK:
        raise IqaError(st, "iqa_probe_read_timeline", _lib.load().iqa_probe_last_hip_error())


def merge_tiles(sums: torch.Tensor, f: int, *, C1: float = C_DEFAULT, C2: float = C_DEFAULT,
                C: float = C_DEFAULT, D: Optional[float] = None, stream=None) -> TileResult:
    """Eq. (3)/(4): merge f x f blocks of tiles (given by their (n, 4) sums
    from ``iqa_tiles(..., sums=True)``) into larger tiles."""
    if sums.dtype != torch.float32 or sums.dim() != 2 or sums.shape[1] != 4 or \
            not sums.is_contiguous():
        raise ValueError("sums must be a contiguous (n, 4) float32 tensor")
    ns = int(round(sums.shape[0] ** 0.5))
    if ns * ns != sums.shape[0]:
        raise ValueError("sums must hold a square number of tiles")
    if D is None:
        D = default_D(C1)
    npar = ns // f if f > 0 and ns % f == 0 else 0
    dev = sums.device
    lo = torch.empty(npar, npar, device=dev)
    ao = torch.empty(npar, npar, device=dev)
    so = torch.empty(npar * npar, 4, device=dev)
    with torch.cuda.device(dev):
        st = _lib.load().iqa_merge_tiles(sums.data_ptr(), ns, f, D, C2, C, lo.data_ptr(),
                                         ao.data_ptr(), so.data_ptr(), _stream_handle(dev, stream))
    _lib.check(st, "iqa_merge_tiles")
    _mark_used(stream, lo, ao, so)
    return TileResult(lo, ao, so)


def pyramid(x: torch.Tensor, y: torch.Tensor, NT: int, *, C1: float = C_DEFAULT,
            C2: float = C_DEFAULT, C: float = C_DEFAULT, D: Optional[float] = None,
            stream=None) -> list:
    """Multi-scale IQA matrices: tiles of NT, 2NT, 4NT, ... up to the largest
    power-of-two multiple of NT that divides N (the whole image when N/NT is a
    power of two).  One fused pass over the images, then a chain of merges."""
    levels = [iqa_tiles(x, y, NT, C1=C1, C2=C2, C=C, D=D, sums=True, stream=stream)]
    ns = x.shape[0] // NT
    while ns % 2 == 0:
        levels.append(merge_tiles(levels[-1].sums, 2, C1=C1, C2=C2, C=C, D=D, stream=stream))
        ns //= 2
    return levels
