"""The measurement entry points: the timeline launch computes the same bits
as the product launch and writes sane stamps; the probes read what they are
given."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import _lib, default_cfg, iqa_tiles, synth
from paper_2501_10653_amd.iqa import (launch_workgroups, probe_empty, probe_read,
                                     probe_read_timeline, tiles_timeline)
from tests.gpu_util import requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("N,NT,ks", [(2048, 64, None), (1024, 256, None), (512, 128, 4),
                                     (600, 24, None)])
def test_timeline_matches_product_launch(N, NT, ks):
    rng = np.random.default_rng(N + NT)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    cfg = default_cfg(N, NT, xd, yd)
    if ks is not None:
        cfg["ksplit"] = ks
    ref = iqa_tiles(xd, yd, NT, cfg=cfg)
    nwg = launch_workgroups(N, NT, cfg)
    stamps = torch.zeros(nwg * 8, dtype=torch.int64, device="cuda")
    got = tiles_timeline(xd, yd, NT, cfg, stamps)
    torch.cuda.synchronize()
    assert same(ref.lisi, got.lisi) and same(ref.auglisi, got.auglisi)
    st = stamps.view(nwg, 8).cpu().numpy()
    entry, first, last, end = st[:, 0], st[:, 1], st[:, 2], st[:, 3]
    assert (entry > 0).all()
    assert (entry <= first).all() and (first <= last).all() and (last <= end).all()
    assert (end - entry).max() < _lib.load().iqa_wall_clock_khz() * 10   # under 10 ms
    part = st[:, 7] & 0xFFFFFFFF
    last = st[:, 7] >> 32
    assert sorted(st[:, 6] * cfg["ksplit"] + part) == list(range(nwg))
    groups = nwg // cfg["ksplit"]
    if cfg["ksplit"] == 1 or nwg <= 1024:
        # exactly one finishing workgroup per tile group (the last part, with
        # a split finished within the launch)
        assert sorted(st[last == 1, 6]) == list(range(groups))
    else:
        # a larger split launch leaves the adding to its combine launch
        assert not last.any()


def test_probe_read_sums_what_it_reads():
    n = 1 << 22
    buf = torch.ones(n, device="cuda")
    for mode in (_lib.PROBE_READ_REGS, _lib.PROBE_READ_REGS_STRUCT, _lib.PROBE_READ_LDS):
        for blocks, threads, loads in ((256, 256, 8), (1024, 512, 4), (97, 64, 32)):
            out = torch.zeros(blocks, device="cuda")
            probe_read(buf, out, threads, loads, mode)
            torch.cuda.synchronize()
            assert float(out.double().sum()) == float(n), (mode, blocks, threads, loads)
    probe_empty(1, 64)
    probe_empty(512, 1024)
    torch.cuda.synchronize()


@pytest.mark.parametrize("blocks,threads,loads", [(256, 512, 4), (97, 64, 32), (1024, 256, 8)])
def test_probe_read_timeline_sums_like_the_read_and_stamps_in_order(blocks, threads, loads):
    n = 1 << 22
    rng = np.random.default_rng(blocks)
    buf = torch.from_numpy(rng.random(n, dtype=np.float32)).cuda()
    ref = torch.zeros(blocks, device="cuda")
    probe_read(buf, ref, threads, loads, _lib.PROBE_READ_REGS)
    out = torch.zeros(blocks, device="cuda")
    stamps = torch.zeros(blocks * 8, dtype=torch.int64, device="cuda")
    probe_read_timeline(buf, out, threads, loads, stamps)
    torch.cuda.synchronize()
    assert same(ref, out)      # the same loads, added in the same order
    st = stamps.view(blocks, 8).cpu().numpy()
    entry, first, last, end = st[:, 0], st[:, 1], st[:, 2], st[:, 3]
    assert (entry > 0).all()
    assert (entry <= first).all() and (first <= last).all() and (last <= end).all()
    assert (st[:, 6] == np.arange(blocks)).all() and (st[:, 7] == 1 << 32).all()
    assert (st[:, 4] & 0xF < 8).all()


def test_probe_read_timeline_refuses_a_short_stamp_buffer():
    buf = torch.ones(1 << 16, device="cuda")
    out = torch.zeros(64, device="cuda")
    stamps = torch.zeros(64 * 8 - 1, dtype=torch.int64, device="cuda")
    with pytest.raises(_lib.IqaError) as e:
        probe_read_timeline(buf, out, 256, 4, stamps)
    assert e.value.status == 2          # IQA_ERR_SHAPE, before any launch
