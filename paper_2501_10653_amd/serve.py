"""Python handle on the library's continuous-batching server (iqa_server_*).

The scheduler is native (a C++ thread inside libiqa_hip.so); this module only
marshals references, requests and completions.  Typical use::

    srv = Server(budget_bytes=8 << 30)
    r = srv.add_reference(ref_tensor)                 # resident on the device
    req = srv.request(snapshot_tensor, r, NT=64)      # allocates its outputs
    srv.submit([req]); srv.drain()
    req.lisi, req.auglisi                             # (N/NT, N/NT) results
"""

from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import Completion, LaunchCfg, Request, ServerOpts, ServerStats
from .iqa import C_DEFAULT, default_D


def serve_cfg(N: int, NT: int) -> dict:
    """Per-pair geometry the server uses for (N, NT): a served request's
    results are bitwise ``iqa_tiles(..., cfg=serve_cfg(N, NT))``."""
    c = LaunchCfg()
    _lib.check(_lib.load().iqa_serve_cfg(N, NT, ctypes.byref(c)), "iqa_serve_cfg")
    return c.as_dict()


class ServedRequest:
    """One request with its own output tensors (kept alive by this object).

    ``ready`` is the event the request's batch waits for on the device before
    it reads the snapshot or writes the outputs (None: no wait)."""

    def __init__(self, snapshot: torch.Tensor, ref_id: int, NT: int, N: int, tag: int,
                 sums: bool = False, host: bool = False,
                 ready: Optional[torch.cuda.Event] = None):
        ns = N // NT if NT > 0 and N % NT == 0 else 0
        dev = torch.device("cuda", torch.cuda.current_device()) if host else snapshot.device
        self.snapshot = snapshot
        self.lisi = torch.empty(ns, ns, device=dev)
        self.auglisi = torch.empty(ns, ns, device=dev)
        self.sums = torch.empty(ns * ns, 4, device=dev) if sums else None
        if ready is True:
            # after the outputs' allocation on the current stream (and whatever
            # that stream still does with their memory, or with the snapshot)
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(dev))
        self.ready = ready or None
        self.c = Request(None if host else snapshot.data_ptr(),
                         snapshot.data_ptr() if host else None,
                         self.lisi.data_ptr(), self.auglisi.data_ptr(),
                         self.sums.data_ptr() if sums else None, NT, ref_id, 0, tag,
                         self.ready.cuda_event if self.ready is not None else None)
        self.NT = NT
        self.ref_id = ref_id
        self.tag = tag


class Server:
    """A continuous-batching server on the current HIP device.

    budget_bytes      admission cap: bytes held by admitted, unfinished requests
                      (a request holds its snapshot plus its outputs).
    streams           launch slots, i.e. batches in flight (1..16).
    max_batch         requests per launch.
    waves             persistent waves per launch (0: the tuned default).
    host_arena_bytes  per slot: device room for snapshots given in pinned host
                      memory (0: device snapshots only).
    C1, C2, C, D      the Eq. 1 / Eq. 2 constants of every request.
    idle_spin_us      how long the scheduler keeps polling after its last work
                      before it sleeps (polling occupies one CPU core; a wake-up
                      from sleep costs several microseconds of latency).

    The server holds every submitted request (its snapshot and its output
    tensors) until its completion has been seen: returned by :meth:`poll`, or
    covered by a :meth:`drain` that succeeded, or by :meth:`close`.  A caller
    may drop its own reference right after :meth:`submit` without the device
    writing into memory that torch has handed to another tensor.
    """

    def __init__(self, budget_bytes: int, *, streams: int = 4, max_batch: int = 512,
                 waves: int = 0, host_arena_bytes: int = 0, C1: float = C_DEFAULT,
                 C2: float = C_DEFAULT, C: float = C_DEFAULT, D: Optional[float] = None,
                 idle_spin_us: float = 1000.0):
        if D is None:
            D = default_D(C1)
        self.opts = ServerOpts(int(budget_bytes), int(host_arena_bytes), int(waves),
                               int(streams), int(max_batch), D, C1, C2, C,
                               int(idle_spin_us * 1000))
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self._lib.iqa_server_create(ctypes.byref(self.opts), ctypes.byref(h)),
                   "iqa_server_create")
        self.h = h
        self.refs: List[torch.Tensor] = []
        self._next_tag = 0
        # submitted requests whose completion has not been seen, by tag (FIFO
        # per tag: tags chosen by the caller need not be unique)
        self._held: Dict[int, List[ServedRequest]] = {}

    def _hold(self, reqs: Sequence[ServedRequest]) -> None:
        for r in reqs:
            self._held.setdefault(r.tag, []).append(r)

    def _release(self, comps: List[dict]) -> None:
        for c in comps:
            held = self._held.get(c["tag"])
            if held:
                held.pop(0)
                if not held:
                    del self._held[c["tag"]]

    def add_reference(self, ref: torch.Tensor) -> int:
        if ref.dtype != torch.float32 or ref.dim() != 2 or ref.shape[0] != ref.shape[1] or \
                not ref.is_contiguous() or ref.device.type != "cuda":
            raise ValueError("reference must be a contiguous N x N float32 device tensor")
        rid = ctypes.c_int32(-1)
        _lib.check(self._lib.iqa_server_add_reference(self.h, ref.data_ptr(), ref.shape[0],
                                                      ctypes.byref(rid)),
                   "iqa_server_add_reference")
        self.refs.append(ref)
        return int(rid.value)

    def request(self, snapshot: torch.Tensor, ref_id: int, NT: int, *, sums: bool = False,
                tag: Optional[int] = None, ready=True) -> ServedRequest:
        """A request for `snapshot` (device tensor, or pinned host tensor) vs
        reference `ref_id`, with freshly allocated outputs.

        The server's streams are not ordered after the caller's.  ``ready``
        orders the request's batch after the caller's work: True (default)
        records an event on the current stream once the outputs are allocated,
        which covers a snapshot produced on that stream; a ``torch.cuda.Event``
        recorded by the caller (e.g. on the stream that produced the snapshot)
        is used as given; False means no wait, for a caller that has
        synchronised the device (or the producing streams) before submitting."""
        if tag is None:
            tag = self._next_tag
            self._next_tag += 1
        host = snapshot.device.type == "cpu"
        if host and not snapshot.is_pinned():
            raise ValueError("host snapshots must be in pinned memory")
        return ServedRequest(snapshot, ref_id, NT, self.refs[ref_id].shape[0], tag, sums, host,
                             ready=ready)

    def submit(self, reqs: Sequence[ServedRequest]) -> None:
        arr = (Request * len(reqs))(*[r.c for r in reqs])
        _lib.check(self._lib.iqa_server_submit(self.h, arr, len(reqs)), "iqa_server_submit")
        self._hold(reqs)

    def poll(self, max_n: int = 4096) -> List[dict]:
        """Completions not yet returned (at most max_n), in completion order;
        the requests they name are no longer held by the server."""
        buf = (Completion * max_n)()
        n = self._lib.iqa_server_poll(self.h, buf, max_n)
        comps = [_completion(buf[i]) for i in range(n)]
        self._release(comps)
        return comps

    def drain(self, timeout_s: float = 60.0) -> None:
        """Wait until every submitted request has completed (their completions
        stay available to :meth:`poll`)."""
        _lib.check(self._lib.iqa_server_drain(self.h, int(timeout_s * 1000)), "iqa_server_drain")
        self._held.clear()

    def stats(self) -> dict:
        st = ServerStats()
        _lib.check(self._lib.iqa_server_get_stats(self.h, ctypes.byref(st)), "iqa_server_stats")
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_ if k != "reserved"}

    def replay(self, reqs: Sequence[ServedRequest], arrival_ns: np.ndarray,
               timeout_s: float = 120.0) -> List[dict]:
        """Open-loop replay: request i is submitted at arrival_ns[i] after the
        start; returns the completions (times relative to the start)."""
        n = len(reqs)
        arr = (Request * n)(*[r.c for r in reqs])
        times = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        out = (Completion * n)()
        st = self._lib.iqa_server_replay(self.h, arr,
                                         times.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         n, out, int(timeout_s * 1000))
        if st != 0:
            # timed out: some of these may still be queued or running
            self._hold(reqs)
        _lib.check(st, "iqa_server_replay")
        return [_completion(out[i]) for i in range(n)]

    def close(self) -> None:
        """Finish all submitted work and free the server."""
        if self.h:
            _lib.check(self._lib.iqa_server_destroy(self.h), "iqa_server_destroy")
            self.h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def _completion(c: Completion) -> dict:
    return {"tag": int(c.tag), "status": int(c.status), "t_submit_ns": int(c.t_submit_ns),
            "t_admit_ns": int(c.t_admit_ns), "t_launch_ns": int(c.t_launch_ns),
            "t_done_ns": int(c.t_done_ns), "t_poll_ns": int(c.t_poll_ns)}


def latency_summary(comps: List[dict]) -> dict:
    """Latency from submission to the caller's poll returning the completion
    (p50_us, p99_us, ...), and to the scheduler seeing the batch complete
    (p50_done_us, p99_done_us); throughput over the span from the first
    submission to the last poll."""
    ok = [c for c in comps if c["status"] == 0]
    lat = np.array([c["t_poll_ns"] - c["t_submit_ns"] for c in ok], dtype=np.float64) / 1e3
    done = np.array([c["t_done_ns"] - c["t_submit_ns"] for c in ok], dtype=np.float64) / 1e3
    if lat.size == 0:
        return {"completed": 0}
    span = (max(c["t_poll_ns"] for c in ok) - min(c["t_submit_ns"] for c in ok)) / 1e9
    return {"completed": len(ok), "failed": len(comps) - len(ok),
            "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "max_us": float(lat.max()), "mean_us": float(lat.mean()),
            "p50_done_us": float(np.percentile(done, 50)),
            "p99_done_us": float(np.percentile(done, 99)),
            "throughput_rps": len(ok) / span if span > 0 else float("nan"), "span_s": span}
