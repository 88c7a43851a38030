"""The continuous-batching server: every result equals the same request served
alone and the single-pair launch with the batch geometry (bitwise), the HBM
budget bounds the bytes in flight, oversized requests are rejected, and an
open-loop Poisson replay completes with correct results."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import iqa_tiles, synth
from paper_2501_10653_amd.serve import Server, latency_summary, serve_cfg
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.fixture(scope="module")
def world():
    """Four small references (N 256/512) with two snapshots each."""
    specs = synth.serving_references(count=4, Ns=(256, 512), seed=5)
    refs, snaps = [], []
    for sp in specs:
        x, _, _ = synth.make_pair(sp)
        refs.append((x, to_dev(x)))
        snaps.append([(s, to_dev(s)) for s in (synth.make_snapshot(sp, k) for k in range(2))])
    return specs, refs, snaps


def make_server(refs, **kw):
    srv = Server(budget_bytes=kw.pop("budget", 1 << 30), **kw)
    ids = [srv.add_reference(d) for _, d in refs]
    return srv, ids


def test_alone_equals_mix_equals_single_launch(world):
    specs, refs, snaps = world
    rng = np.random.default_rng(3)
    plan = [(int(rng.integers(4)), int(rng.integers(2)), int(rng.choice([16, 32, 64])))
            for _ in range(60)]
    srv, ids = make_server(refs)
    mix = [srv.request(snaps[r][k][1], ids[r], NT) for r, k, NT in plan]
    srv.submit(mix)
    srv.drain()
    comps = srv.poll(1000)
    assert len(comps) == len(mix) and all(c["status"] == 0 for c in comps)
    st = srv.stats()
    assert st["batches"] >= 1 and st["completed"] == len(mix)
    srv.close()
    for (r, k, NT), req in list(zip(plan, mix))[:12]:
        alone_srv, aid = make_server(refs)
        alone = alone_srv.request(snaps[r][k][1], aid[r], NT)
        alone_srv.submit([alone])
        alone_srv.drain()
        alone_srv.close()
        assert same(alone.lisi, req.lisi) and same(alone.auglisi, req.auglisi)
        N = refs[r][1].shape[0]
        single = iqa_tiles(snaps[r][k][1], refs[r][1], NT, cfg=serve_cfg(N, NT))
        torch.cuda.synchronize()
        assert same(single.lisi, req.lisi) and same(single.auglisi, req.auglisi)


@pytest.mark.parametrize("max_batch", [1, 3, 16, 17])
def test_servers_of_every_batch_limit_warm_up_and_serve(world, max_batch):
    """Creation runs every launch form the batch limit allows once, on a zero
    pair (1, 4 and 16 inline descriptors, a descriptor table); the server then
    serves as usual, every result bitwise the single launch."""
    specs, refs, snaps = world
    srv, ids = make_server(refs, max_batch=max_batch)
    plan = [(r % 4, (r // 4) % 2) for r in range(20)]
    reqs = [srv.request(snaps[r][k][1], ids[r], 32) for r, k in plan]
    srv.submit(reqs)
    srv.drain()
    comps = srv.poll(100)
    st = srv.stats()
    srv.close()
    assert len(comps) == 20 and all(c["status"] == 0 for c in comps)
    assert st["max_batch"] <= max_batch
    for (r, k), req in zip(plan, reqs):
        N = refs[r][1].shape[0]
        single = iqa_tiles(snaps[r][k][1], refs[r][1], 32, cfg=serve_cfg(N, 32))
        torch.cuda.synchronize()
        assert same(single.lisi, req.lisi) and same(single.auglisi, req.auglisi)


def test_results_match_oracle(world):
    specs, refs, snaps = world
    srv, ids = make_server(refs)
    reqs = [srv.request(snaps[r][0][1], ids[r], 32, sums=True) for r in range(4)]
    srv.submit(reqs)
    srv.drain()
    srv.close()
    for r, req in enumerate(reqs):
        assert_parity(req, oracle_for(snaps[r][0][0], refs[r][0], 32), what=f"ref {r}")


def test_budget_bounds_bytes_in_flight(world):
    specs, refs, snaps = world
    one = 4 * 512 * 512 + 8 * 16 * 16     # largest request: 512^2 snapshot, 32-tiles
    srv, ids = make_server(refs, budget=one + 1000, streams=2)
    reqs = [srv.request(snaps[r % 4][0][1], ids[r % 4], 32) for r in range(16)]
    srv.submit(reqs)
    srv.drain()
    st = srv.stats()
    srv.close()
    assert st["completed"] == 16 and st["peak_in_flight_bytes"] <= one + 1000
    # a 512^2 request never shares the budget with another one
    assert st["batches"] >= 8


def test_oversized_and_invalid_requests_rejected(world):
    specs, refs, snaps = world
    srv, ids = make_server(refs, budget=1 << 20)   # 1 MiB: a 512^2 snapshot is 1 MiB + outputs
    big = ids[[i for i, (_, d) in enumerate(refs) if d.shape[0] == 512][0]]
    small = ids[[i for i, (_, d) in enumerate(refs) if d.shape[0] == 256][0]]
    r_big = srv.request(snaps[big][0][1], big, 64)
    r_bad = srv.request(snaps[small][0][1], small, 48)      # 256 % 48 != 0
    r_ok = srv.request(snaps[small][0][1], small, 64)
    srv.submit([r_big, r_bad, r_ok])
    srv.drain()
    comps = {c["tag"]: c["status"] for c in srv.poll()}
    srv.close()
    assert comps[r_big.tag] == 8      # IQA_ERR_BUDGET
    assert comps[r_bad.tag] == 2      # IQA_ERR_SHAPE
    assert comps[r_ok.tag] == 0


def test_host_snapshots_equal_device_snapshots(world):
    specs, refs, snaps = world
    srv, ids = make_server(refs, host_arena_bytes=8 << 20)
    dev_reqs, host_reqs = [], []
    for r in range(4):
        hs = torch.from_numpy(snaps[r][1][0]).pin_memory()
        dev_reqs.append(srv.request(snaps[r][1][1], ids[r], 64))
        host_reqs.append(srv.request(hs, ids[r], 64))
    srv.submit(dev_reqs + host_reqs)
    srv.drain()
    srv.close()
    for a, b in zip(dev_reqs, host_reqs):
        assert same(a.lisi, b.lisi) and same(a.auglisi, b.auglisi)


def test_poisson_replay(world):
    specs, refs, snaps = world
    rng = np.random.default_rng(9)
    srv, ids = make_server(refs, max_batch=64)
    reqs = []
    for i in range(400):
        r = int(rng.integers(4))
        reqs.append(srv.request(snaps[r][i % 2][1], ids[r], int(rng.choice([32, 64]))))
    arrivals = synth.poisson_arrivals(rate=20000, count=len(reqs), seed=1)
    comps = srv.replay(reqs, arrivals)
    srv.close()
    summ = latency_summary(comps)
    assert summ["completed"] == 400 and summ["failed"] == 0
    assert 0 < summ["p50_us"] <= summ["p99_us"]
    for c in comps:
        assert c["t_submit_ns"] <= c["t_admit_ns"] <= c["t_launch_ns"] <= c["t_done_ns"]
    # spot-check results of the replay against the oracle
    for req in reqs[:5]:
        r = req.ref_id
        k = [i for i in range(2) if snaps[r][i][1].data_ptr() == req.snapshot.data_ptr()][0]
        assert_parity(req, oracle_for(snaps[r][k][0], refs[r][0], req.NT), what="replay")


def test_server_holds_dropped_requests_until_completion_is_seen(world):
    """A request the caller drops right after submit stays alive (snapshot and
    outputs) until its completion has been seen: by poll, or by drain."""
    import gc
    import time
    import weakref
    specs, refs, snaps = world
    with make_server(refs[:1])[0] as srv:
        # completion seen through poll
        req = srv.request(snaps[0][0][1], 0, 32)
        w = weakref.ref(req)
        srv.submit([req])
        del req
        gc.collect()
        assert w() is not None
        comps, deadline = [], time.time() + 30
        while not comps and time.time() < deadline:
            comps += srv.poll()
        assert len(comps) == 1 and comps[0]["status"] == 0
        gc.collect()
        assert w() is None
        # completion covered by drain
        req = srv.request(snaps[0][1][1], 0, 64)
        w = weakref.ref(req)
        srv.submit([req])
        del req
        gc.collect()
        assert w() is not None
        srv.drain()
        gc.collect()
        assert w() is None
        assert len(srv.poll()) == 1


def test_ready_event_orders_batch_after_producer_stream(world):
    """A snapshot written by a torch op on a side stream right before submit
    (behind a long fill on that stream) is read only after the write: the
    request carries an event recorded on the side stream, and its result
    equals the single-pair launch on the finished snapshot, bitwise."""
    specs, refs, snaps = world
    r = 3
    N = refs[r][1].shape[0]
    side = torch.cuda.Stream()
    busy = torch.empty(256 << 20, device="cuda")       # 1 GiB: a fill of ~0.2 ms
    srv, ids = make_server(refs)
    reqs, dsts = [], []
    for k in range(8):
        dst = torch.zeros(N, N, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            busy.fill_(float(k))
            dst.copy_(snaps[r][k % 2][1])
            dst.record_stream(side)
            ev = torch.cuda.Event()
            ev.record(side)
        req = srv.request(dst, ids[r], 64, ready=ev)
        srv.submit([req])
        reqs.append((req, k % 2))
        dsts.append(dst)
    srv.drain()
    comps = srv.poll(100)
    srv.close()
    assert len(comps) == 8 and all(c["status"] == 0 for c in comps)
    torch.cuda.synchronize()
    single = [iqa_tiles(snaps[r][k][1], refs[r][1], 64, cfg=serve_cfg(N, 64)) for k in range(2)]
    torch.cuda.synchronize()
    for req, k in reqs:
        assert same(single[k].lisi, req.lisi) and same(single[k].auglisi, req.auglisi)


def test_completion_times_are_ordered_to_the_poll(world):
    specs, refs, snaps = world
    srv, ids = make_server(refs)
    reqs = [srv.request(snaps[r % 4][0][1], ids[r % 4], 32) for r in range(32)]
    srv.submit(reqs)
    srv.drain()
    comps = srv.poll(100)
    srv.close()
    assert len(comps) == 32
    for c in comps:
        assert c["t_submit_ns"] <= c["t_admit_ns"] <= c["t_launch_ns"] <= c["t_done_ns"]
        assert c["t_done_ns"] <= c["t_poll_ns"]
    summ = latency_summary(comps)
    assert summ["p50_done_us"] <= summ["p50_us"]
