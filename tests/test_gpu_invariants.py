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
