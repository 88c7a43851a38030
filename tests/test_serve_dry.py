"""The serving scheduler's policy on the CPU, through the dry-run server: it
admits, batches and retires exactly like the GPU server but launches nothing
and completes a batch of b bytes after fixed + b / bandwidth nanoseconds."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_2501_10653_amd import _lib, synth
from paper_2501_10653_amd._lib import Completion, Request, ServerOpts, ServerStats

FAKE = 1 << 24           # aligned stand-ins for device pointers, never dereferenced
C6 = 1e-6


class Dry:
    def __init__(self, budget=1 << 40, streams=2, max_batch=64, arena=0, fixed_ns=20000,
                 bytes_per_ns=5000.0, refs=(1024, 2048, 4096)):
        self.lib = _lib.load()
        opts = ServerOpts(budget, arena, 0, streams, max_batch, C6 / 2, C6, C6, C6)
        self.h = ctypes.c_void_p()
        st = self.lib.iqa_server_create_dry(ctypes.byref(opts), fixed_ns, bytes_per_ns,
                                            ctypes.byref(self.h))
        assert st == 0
        self.N = list(refs)
        for N in refs:
            rid = ctypes.c_int32()
            assert self.lib.iqa_server_add_reference(self.h, FAKE, N, ctypes.byref(rid)) == 0

    def req(self, ref, NT, tag, host=False, out=True):
        return Request(None if host else FAKE, FAKE if host else None,
                       FAKE if out else None, FAKE if out else None, None, NT, ref, 0, tag)

    def submit(self, reqs):
        arr = (Request * len(reqs))(*reqs)
        assert self.lib.iqa_server_submit(self.h, arr, len(reqs)) == 0

    def drain(self, ms=20000):
        assert self.lib.iqa_server_drain(self.h, ms) == 0

    def poll(self):
        buf = (Completion * 100000)()
        n = self.lib.iqa_server_poll(self.h, buf, 100000)
        return [buf[i] for i in range(n)]

    def stats(self):
        st = ServerStats()
        assert self.lib.iqa_server_get_stats(self.h, ctypes.byref(st)) == 0
        return st

    def replay(self, reqs, arrivals):
        arr = (Request * len(reqs))(*reqs)
        t = np.ascontiguousarray(arrivals, np.int64)
        out = (Completion * len(reqs))()
        st = self.lib.iqa_server_replay(self.h, arr, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        len(reqs), out, 60000)
        assert st == 0
        return [out[i] for i in range(len(reqs))]

    def close(self):
        assert self.lib.iqa_server_destroy(self.h) == 0


def cost(N, NT):
    ns = N // NT
    return 4 * N * N + 8 * ns * ns


def test_everything_completes_in_order_with_consistent_times():
    d = Dry()
    reqs = [d.req(i % 3, 64, i) for i in range(200)]
    d.submit(reqs)
    d.drain()
    comps = d.poll()
    d.close()
    assert sorted(c.tag for c in comps) == list(range(200))
    assert all(c.status == 0 for c in comps)
    for c in comps:
        assert c.t_submit_ns <= c.t_admit_ns <= c.t_launch_ns <= c.t_done_ns
    # admission is FIFO: admit times are non-decreasing in submission order
    admit = {c.tag: c.t_admit_ns for c in comps}
    assert all(admit[i] <= admit[i + 1] for i in range(199))


def test_budget_bounds_bytes_in_flight_and_forces_small_batches():
    big = cost(4096, 64)
    d = Dry(budget=big + cost(1024, 64) - 1)         # a 4096 request never shares
    d.submit([d.req(i % 3, 64, i) for i in range(60)])
    d.drain()
    st = d.stats()
    d.close()
    assert st.completed == 60 and st.rejected == 0
    assert st.peak_in_flight_bytes <= big + cost(1024, 64) - 1
    assert st.batches >= 20                            # one per 4096^2 request at least


def test_oversized_and_invalid_requests_are_rejected():
    d = Dry(budget=cost(2048, 64))
    d.submit([d.req(2, 64, 0),          # 4096^2: over budget
              d.req(0, 48, 1),          # 1024 % 48 != 0
              d.req(0, 30, 2),          # NT % 4 != 0
              d.req(7, 64, 3),          # no such reference
              d.req(0, 64, 4, out=False),
              d.req(1, 64, 5)])         # fits
    d.drain()
    got = {c.tag: c.status for c in d.poll()}
    st = d.stats()
    d.close()
    assert got == {0: 8, 1: 2, 2: 2, 3: 6, 4: 1, 5: 0}
    assert st.rejected == 5 and st.completed == 6


def test_host_snapshots_need_arena_room():
    d = Dry(arena=4 * 2048 * 2048)
    d.submit([d.req(2, 64, 0, host=True),      # 4096^2 host snapshot: no room
              d.req(1, 64, 1, host=True)])     # 2048^2: fits the arena
    d.drain()
    got = {c.tag: c.status for c in d.poll()}
    d.close()
    assert got == {0: 8, 1: 0}


def test_continuous_batching_under_load():
    """With one slot and a slow service, requests that arrive while a batch
    runs are admitted together into the next launch."""
    d = Dry(streams=1, max_batch=1000, fixed_ns=2_000_000, bytes_per_ns=1e9)
    reqs = [d.req(0, 64, i) for i in range(300)]
    arrivals = synth.poisson_arrivals(rate=50000, count=300, seed=4)
    comps = d.replay(reqs, arrivals)
    st = d.stats()
    d.close()
    assert len(comps) == 300 and all(c.status == 0 for c in comps)
    assert st.max_batch >= 20 and st.batches < 100
    # every batch's launch happens only after the previous batch completed
    launches = sorted({c.t_launch_ns for c in comps})
    dones = sorted({c.t_done_ns for c in comps})
    assert all(launches[i + 1] >= dones[i] for i in range(len(dones) - 1))


def test_two_slots_overlap_batches():
    d = Dry(streams=2, max_batch=4, fixed_ns=1_000_000, bytes_per_ns=1e9)
    d.submit([d.req(0, 64, i) for i in range(16)])
    d.drain()
    comps = d.poll()
    d.close()
    spans = sorted({(c.t_launch_ns, c.t_done_ns) for c in comps})
    overlaps = sum(1 for a, b in zip(spans, spans[1:]) if b[0] < a[1])
    assert overlaps >= 1


def test_latency_grows_only_past_capacity():
    """A modelled service of 1 ms per batch plus 50 GB/s (168 us per 1024^2
    request) serves ~11k req/s with two slots.  At 1k req/s the p99 latency
    stays near the service time; at 30k req/s requests queue and p99 grows
    many times over (large margins: OS scheduling jitter must not matter)."""
    def p99(rate, count):
        d = Dry(streams=2, max_batch=64, fixed_ns=1_000_000, bytes_per_ns=50.0)
        reqs = [d.req(0, 64, i) for i in range(count)]
        comps = d.replay(reqs, synth.poisson_arrivals(rate, count, seed=5))
        d.close()
        lat = np.array([c.t_done_ns - c.t_submit_ns for c in comps])
        return np.percentile(lat, 99)
    light, heavy = p99(1000, 100), p99(30000, 300)
    assert heavy > 4 * light


def test_dry_options_validated():
    lib = _lib.load()
    opts = ServerOpts(1 << 30, 0, 0, 2, 64, C6 / 2, C6, C6, C6)
    h = ctypes.c_void_p()
    assert lib.iqa_server_create_dry(ctypes.byref(opts), -1, 1.0, ctypes.byref(h)) == 6
    assert lib.iqa_server_create_dry(ctypes.byref(opts), 0, 0.0, ctypes.byref(h)) == 6
