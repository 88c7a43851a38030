"""Eq. (3)/(4) aggregation on the GPU against the oracle's literal Eq. (3)/(4)
merge and against the oracle's direct values on the larger tiles."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2501_10653_amd import iqa_tiles, merge_tiles, pyramid, synth
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def small():
    x, y, _ = synth.make_pair(synth.spec_small())
    return x, y, to_dev(x), to_dev(y)


@pytest.mark.parametrize("f", [1, 2, 4, 16])
def test_merge_vs_oracle_eq34(small, f):
    x, y, xd, yd = small
    NT = 16
    child_gpu = iqa_tiles(xd, yd, NT, sums=True)
    merged = merge_tiles(child_gpu.sums, f)
    torch.cuda.synchronize()
    c = oracle.f32const(1e-6)
    child = oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)
    ora = oracle.merge_tiles(child[0], child[1], child[2], f, c, c)
    assert_parity(merged, ora, what=f"merge f={f}")


def test_whole_image_value(small):
    x, y, xd, yd = small
    res = iqa_tiles(xd, yd, 32, sums=True)
    whole = merge_tiles(res.sums, 8)
    torch.cuda.synchronize()
    assert whole.lisi.shape == (1, 1)
    assert_parity(whole, oracle_for(x, y, 256), what="whole image")


def test_pyramid_paper_shape():
    x, y, _ = synth.make_pair(synth.spec_paper_shape())
    levels = pyramid(to_dev(x), to_dev(y), 64)
    torch.cuda.synchronize()
    assert [lv.lisi.shape[0] for lv in levels] == [32, 16, 8, 4, 2, 1]
    for i, lv in enumerate(levels):
        assert_parity(lv, oracle_for(x, y, 64 << i), what=f"level {i}")


def test_merge_of_split_tiles_ragged_sizes():
    rng = np.random.default_rng(12)
    x, y = synth.random_pair(600, rng, neg_frac=0.3, nan_frac=0.02, scale=2.0)
    res = iqa_tiles(to_dev(x), to_dev(y), 24, sums=True)
    for f in (5, 25):
        m = merge_tiles(res.sums, f)
        torch.cuda.synchronize()
        assert_parity(m, oracle_for(x, y, 24 * f), what=f"600/24 f={f}")
