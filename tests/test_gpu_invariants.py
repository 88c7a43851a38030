"""Bitwise properties of the HIP path that follow from the method and from the
kernel's fixed reduction order, plus every instantiated launch configuration
against the oracle."""

from __future__ import annotations

import itertools

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import (IqaError, auglisi_tiles, check_cfg, default_cfg, iqa_tiles,
                                  lisi_tiles, synth)
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def paper_pair():
    x, y, _ = synth.make_pair(synth.spec_paper_shape())
    return x, y, to_dev(x), to_dev(y)


def fused(xd, yd, NT, **kw):
    r = iqa_tiles(xd, yd, NT, sums=True, **kw)
    torch.cuda.synchronize()
    return r


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_run_to_run_bitwise(paper_pair):
    _, _, xd, yd = paper_pair
    a = fused(xd, yd, 64)
    for _ in range(3):
        b = fused(xd, yd, 64)
        assert same(a.lisi, b.lisi) and same(a.auglisi, b.auglisi) and same(a.sums, b.sums)


@pytest.mark.parametrize("N,NT", [(2048, 64), (1024, 256), (256, 32), (300, 12), (2048, 1024)])
def test_symmetry_bitwise(N, NT):
    rng = np.random.default_rng(N + NT)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    a = fused(xd, yd, NT)
    b = fused(yd, xd, NT)
    assert same(a.lisi, b.lisi) and same(a.auglisi, b.auglisi)
    assert same(a.sums[:, :2], b.sums[:, :2])
    assert same(a.sums[:, 2], b.sums[:, 3]) and same(a.sums[:, 3], b.sums[:, 2])


def test_clamp_invariance_bitwise(paper_pair):
    x, y, xd, yd = paper_pair
    rng = np.random.default_rng(1)
    x2 = x.copy()
    neg = x2 <= 0
    x2[neg] = rng.choice(np.array([-5.0, -1e-20, -0.0, 0.0, np.nan], np.float32),
                         size=int(neg.sum()))
    a = fused(xd, yd, 64)
    b = fused(to_dev(x2), yd, 64)
    assert same(a.lisi, b.lisi) and same(a.auglisi, b.auglisi) and same(a.sums, b.sums)


def test_tile_locality_bitwise(paper_pair):
    x, y, xd, yd = paper_pair
    base = fused(xd, yd, 64)
    for r, c in [(0, 0), (70, 1500), (2047, 2047), (1024, 63)]:
        x2 = x.copy()
        x2[r, c] += np.float32(0.25)
        got = fused(to_dev(x2), yd, 64)
        diff = ((got.lisi != base.lisi) | (got.auglisi != base.auglisi)).flatten()
        idx = torch.nonzero(diff).flatten().tolist()
        assert idx == [(r // 64) * 32 + c // 64], (r, c, idx)


@pytest.mark.parametrize("N,NT", [(2048, 64), (1024, 256), (300, 12), (1000, 8), (2048, 512)])
def test_separate_entry_points_equal_fused_bitwise(N, NT):
    rng = np.random.default_rng(N * 3 + NT)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    a = fused(xd, yd, NT)
    l = lisi_tiles(xd, yd, NT)
    g = auglisi_tiles(xd, yd, NT)
    torch.cuda.synchronize()
    assert same(a.lisi, l) and same(a.auglisi, g)


def all_configs(N, NT):
    """Every instantiated (vec, waves, unroll) with a spread of rp and ksplit."""
    out = []
    combos = [(4, w, u) for w in (1, 2, 4, 8) for u in (4, 8)] + \
        [(4, 16, 4), (2, 1, 4), (2, 4, 4), (1, 1, 4), (1, 4, 4)]
    for vec, waves, unroll in combos:
        if NT % vec:
            continue
        lpt = NT // vec
        seg = min(64, 1 << (lpt - 1).bit_length())
        for seg_ in {seg, max(1, seg // 2)}:
            for rp, ks in itertools.product((1, 2, 4, 64), (1, 2, 8, NT)):
                if seg_ * rp > 64:
                    continue
                cfg = dict(vec=vec, waves=waves, unroll=unroll, seg=seg_, rp=rp, ksplit=ks)
                if check_cfg(N, NT, cfg) == 0 and cfg not in out:
                    out.append(cfg)
    return out


@pytest.mark.parametrize("N,NT", [(2048, 64), (1024, 256), (512, 16), (600, 24)])
def test_every_instantiated_config(N, NT):
    rng = np.random.default_rng(N + 17 * NT)
    x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    ora = oracle_for(x, y, NT)
    cfgs = all_configs(N, NT)
    assert len(cfgs) >= 10
    for cfg in cfgs:
        res = iqa_tiles(xd, yd, NT, sums=True, cfg=cfg)
        torch.cuda.synchronize()
        assert_parity(res, ora, what=str(cfg))


SPLIT_SHAPES = [(1024, 256, None), (512, 512, None), (2048, 1024, None), (256, 128, 4)]


def split_cfg(N, NT, ks):
    cfg = default_cfg(N, NT)
    if ks is not None:
        cfg["ksplit"] = ks
    return cfg


def test_split_shapes_use_split():
    for N, NT, ks in SPLIT_SHAPES:
        cfg = split_cfg(N, NT, ks)
        assert cfg["ksplit"] > 1 and check_cfg(N, NT, cfg) == 0, (N, NT, cfg)


def test_split_workspace_reuse_across_shapes():
    """The per-stream split workspace grows as shapes alternate on one stream,
    and every result stays right."""
    rng = np.random.default_rng(4)
    pairs = {}
    for N, NT, ks in SPLIT_SHAPES:
        x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
        pairs[(N, NT)] = (split_cfg(N, NT, ks), to_dev(x), to_dev(y), oracle_for(x, y, NT))
    for _ in range(2):
        for (N, NT), (cfg, xd, yd, ora) in pairs.items():
            res = fused(xd, yd, NT, cfg=cfg)
            assert_parity(res, ora, what=f"{N}/{NT}")


def test_invalid_arguments_raise():
    xd = torch.zeros(64, 64, device="cuda")
    with pytest.raises(IqaError):
        iqa_tiles(xd, xd, 7)
    with pytest.raises(IqaError):
        iqa_tiles(xd, xd, 8, C1=0.0)
    with pytest.raises(TypeError):
        iqa_tiles(xd.double(), xd.double(), 8)
    with pytest.raises(ValueError):
        iqa_tiles(xd.t(), xd, 8)


# 2048/256 split 64 ways: 64 tile groups x 64 parts x 16 B = 64 KiB of
# partials, more than the 4 KiB a 512/512 launch needs.
GROW_CFG = dict(vec=4, waves=1, unroll=4, seg=64, rp=1, ksplit=64)


def test_graph_replays_with_split_workspace_growth():
    """A captured split-shape launch stays correct across replays even after a
    larger shape grows the stream's workspace (the old buffer is kept), with
    eager work between the replays."""
    from paper_2501_10653_amd import prepare
    rng = np.random.default_rng(21)
    x, y = synth.random_pair(512, rng, neg_frac=0.3, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    cfg = split_cfg(512, 512, None)
    s = torch.cuda.Stream()
    prepare(512, 512, cfg, stream=s)
    out = {"lisi": torch.empty(1, 1, device="cuda"), "auglisi": torch.empty(1, 1, device="cuda")}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        iqa_tiles(xd, yd, 512, out=out, cfg=cfg, stream=s)
    ora = oracle_for(x, y, 512)
    x2, y2 = synth.random_pair(2048, rng, neg_frac=0.3, scale=1.0)
    big = (to_dev(x2), to_dev(y2))
    for rep in range(3):
        out["lisi"].fill_(-1.0)
        out["auglisi"].fill_(-1.0)
        with torch.cuda.stream(s):
            g.replay()
            # eager work on the same stream, growing the workspace on the first pass
            iqa_tiles(big[0], big[1], 256, cfg=GROW_CFG, stream=s)
        torch.cuda.synchronize()
        from paper_2501_10653_amd.iqa import TileResult
        assert_parity(TileResult(out["lisi"], out["auglisi"], None), ora, what=f"replay {rep}")


def test_single_pair_graph_replays_equal_eager(paper_pair):
    _, _, xd, yd = paper_pair
    eager = fused(xd, yd, 64)
    s = torch.cuda.Stream()
    out = {"lisi": torch.empty(32, 32, device="cuda"), "auglisi": torch.empty(32, 32, device="cuda")}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        iqa_tiles(xd, yd, 64, out=out, stream=s)
    for rep in range(3):
        out["lisi"].zero_()
        out["auglisi"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        assert same(out["lisi"], eager.lisi) and same(out["auglisi"], eager.auglisi), rep
