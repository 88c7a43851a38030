"""Split shapes (several workgroups per tile group): determinism, symmetry,
concurrent callers on one stream, and graph replays, against single runs and
the oracle.  Launches of at most 1024 workgroups add their parts by ticket
(the last part to finish adds them); larger ones through a second, combine
launch; both mechanisms are covered."""

from __future__ import annotations

import threading

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import check_cfg, default_cfg, iqa_tiles, synth
from paper_2501_10653_amd.iqa import TileResult
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

# (N, NT, ksplit): the default split shapes of the size sweep's large-tile
# cells, and hand-picked deeper splits (up to one row per workgroup slice).
TICKET_MAX_GRID = 1024
COMBINE = dict(waves=1, unroll=8, ksplit=8)      # 2048^2/128: 2048 workgroups
SHAPES = [(2048, 256, None), (1024, 256, None), (1024, 512, None), (2048, 128, dict(ksplit=8)),
          (512, 512, dict(waves=1, unroll=4, ksplit=128)), (256, 64, dict(ksplit=16)),
          (2048, 128, COMBINE), (4096, 128, dict(waves=1, unroll=8, ksplit=4)),
          (1024, 64, dict(waves=1, unroll=4, ksplit=4))]


def cfg_for(N, NT, over):
    cfg = default_cfg(N, NT)
    if over is not None:
        cfg.update(over)
    assert check_cfg(N, NT, cfg) == 0, (N, NT, cfg)
    return cfg


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def run(xd, yd, NT, cfg, stream=None):
    r = iqa_tiles(xd, yd, NT, sums=True, cfg=cfg, stream=stream)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("N,NT,over", SHAPES)
def test_split_parity_determinism_symmetry(N, NT, over):
    cfg = cfg_for(N, NT, over)
    assert cfg["ksplit"] > 1
    rng = np.random.default_rng(N * 7 + NT)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    a = run(xd, yd, NT, cfg)
    assert_parity(a, oracle_for(x, y, NT), what=f"{N}/{NT} {cfg}")
    for _ in range(5):   # whichever part comes last, the parts add in part order
        b = run(xd, yd, NT, cfg)
        assert same(a.lisi, b.lisi) and same(a.auglisi, b.auglisi) and same(a.sums, b.sums)
    c = run(yd, xd, NT, cfg)
    assert same(a.lisi, c.lisi) and same(a.auglisi, c.auglisi)


def test_both_mechanisms_are_covered():
    from paper_2501_10653_amd.iqa import launch_workgroups
    grids = [launch_workgroups(N, NT, cfg_for(N, NT, over)) for N, NT, over in SHAPES]
    assert min(grids) <= TICKET_MAX_GRID < max(grids)


@pytest.mark.parametrize("use_null_stream", [False, True])
@pytest.mark.parametrize("NT,over", [(256, None), (128, COMBINE)])
def test_two_threads_share_one_stream(use_null_stream, NT, over):
    """Two host threads issue split launches with different inputs on one
    shared stream (a torch stream, or the legacy NULL stream) as fast as they
    can; every result equals the same launch run alone, bitwise (a combine
    launch never reads another call's partials)."""
    N = 2048
    cfg = cfg_for(N, NT, over)
    rng = np.random.default_rng(99)
    inputs = []
    for _ in range(2):
        x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
        inputs.append((x, y, to_dev(x), to_dev(y)))
    stream = None if use_null_stream else torch.cuda.Stream()
    handle = 0 if use_null_stream else stream
    alone = [run(xd, yd, NT, cfg) for _, _, xd, yd in inputs]
    reps = 200
    results = [[None] * reps for _ in range(2)]
    errors = []

    def worker(t):
        try:
            torch.cuda.set_device(0)
            xd, yd = inputs[t][2], inputs[t][3]
            for i in range(reps):
                results[t][i] = iqa_tiles(xd, yd, NT, cfg=cfg, stream=handle)
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for t in range(2):
        for i in range(reps):
            r = results[t][i]
            assert same(r.lisi, alone[t].lisi) and same(r.auglisi, alone[t].auglisi), (t, i)
    assert_parity(alone[0], oracle_for(inputs[0][0], inputs[0][1], NT), what="thread 0")


def test_split_graph_replays_with_eager_split_work_between():
    """A graph of split launches on two inputs, replayed several times with
    eager split launches of other inputs on the same stream in between: every
    replay equals the eager result, bitwise."""
    N, NT = 1024, 256
    cfg = cfg_for(N, NT, None)
    rng = np.random.default_rng(5)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    x2, y2 = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    xd, yd, xd2, yd2 = to_dev(x), to_dev(y), to_dev(x2), to_dev(y2)
    s = torch.cuda.Stream()
    eager = run(xd, yd, NT, cfg, stream=s)
    ns = N // NT
    outs = [{"lisi": torch.empty(ns, ns, device="cuda"),
             "auglisi": torch.empty(ns, ns, device="cuda")} for _ in range(2)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        iqa_tiles(xd, yd, NT, cfg=cfg, out=outs[0], stream=s)
        iqa_tiles(xd, yd, NT, cfg=cfg, out=outs[1], stream=s)
    for rep in range(4):
        for o in outs:
            o["lisi"].fill_(-1.0)
            o["auglisi"].fill_(-1.0)
        with torch.cuda.stream(s):
            g.replay()
            other = iqa_tiles(xd2, yd2, NT, cfg=cfg, stream=s)
        torch.cuda.synchronize()
        for o in outs:
            assert same(o["lisi"], eager.lisi) and same(o["auglisi"], eager.auglisi), rep
        assert_parity(TileResult(other.lisi, other.auglisi, None), oracle_for(x2, y2, NT),
                      what=f"eager between replays {rep}")
