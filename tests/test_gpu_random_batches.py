"""Seeded random batches: 1-40 pairs of mixed sizes (some with N_T % 4 != 0
or unaligned images, which the batch launches one by one), a random
persistent wave count, descriptors inline or in a device table, and for some
shapes a registered geometry of one wave per tile group or of four waves
splitting its rows.  Every pair is checked against the oracle, and every pair
the persistent kernel took is bitwise equal to its single-pair launch with the
batch geometry."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import _lib, iqa_tiles, synth
from paper_2501_10653_amd._lib import LaunchCfg
from paper_2501_10653_amd.batch import Batch, batch_cfg
from tests.gpu_util import assert_parity, oracle_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = 30


def _case(i):
    rng = np.random.default_rng((31, i))
    count = int(rng.integers(1, 41))
    pairs = []
    for _ in range(count):
        NT = int(rng.choice([4, 8, 12, 16, 32, 64, 128, 256, 512, 6, 10]))
        ns = int(rng.integers(1, max(2, 768 // NT) + 1))
        off = int(rng.choice([0, 0, 0, 1]))          # 1: a 4-byte (not 16-byte) aligned image
        pairs.append((NT * ns, NT, off))
    waves = int(rng.choice([4, 64, 512, 2048, 4096, 8192]))
    inline = None if rng.uniform() < 0.7 else False
    # per-(N, N_T) geometries registered for this case: four waves splitting
    # the rows of each tile group, or one wave per group, at a random rp
    geoms = {}
    for N, NT, _ in pairs:
        if NT % 4 == 0 and rng.uniform() < 0.5:
            lpt = NT // 4
            seg = min(64, 1 << (lpt - 1).bit_length())
            rp = int(rng.choice([r for r in (1, 2, 4, 8) if seg * r <= 64]))
            geoms[(N, NT)] = dict(vec=4, waves=int(rng.choice([1, 4])), unroll=8, seg=seg, rp=rp,
                                  ksplit=1)
    return count, pairs, waves, inline, geoms


@pytest.fixture
def tuned():
    lib = _lib.load()
    yield lib
    lib.iqa_tune_clear()


@pytest.mark.parametrize("i", range(CASES))
def test_random_batch(i, tuned):
    count, shapes, waves, inline, geoms = _case(i)
    for (N, NT), cfg in geoms.items():
        assert tuned.iqa_tune_set(N, NT, _lib.TUNE_BATCH, LaunchCfg.from_dict(cfg)) == 0
    rng = np.random.default_rng((32, i))
    dev = torch.device("cuda", 0)
    host, pairs = [], []
    for N, NT, off in shapes:
        x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01)
        bx = torch.empty(N * N + 4, device=dev)
        by = torch.empty(N * N + 4, device=dev)
        xd = bx[off:off + N * N].view(N, N)
        yd = by[off:off + N * N].view(N, N)
        xd.copy_(torch.from_numpy(x))
        yd.copy_(torch.from_numpy(y))
        host.append((x, y, NT))
        pairs.append((xd, yd, NT))
    vec4 = [NT % 4 == 0 and off == 0 for N, NT, off in shapes]
    if inline is None and sum(vec4) > 16:
        inline = False
    b = Batch(pairs, waves=waves, inline=inline)
    print(f"batch {i}: {count} pairs, {b.count} persistent, waves {waves}, inline {b.inline}, "
          f"{sum(c['waves'] == 4 for c in geoms.values())} four-wave geometries", flush=True)
    b.run()
    torch.cuda.synchronize()
    for k, ((x, y, NT), (xd, yd, _), res) in enumerate(zip(host, pairs, b.results)):
        assert_parity(res, oracle_for(x, y, NT), what=f"batch {i} pair {k} N={x.shape[0]} NT={NT}")
        if vec4[k]:
            single = iqa_tiles(xd, yd, NT, cfg=batch_cfg(x.shape[0], NT))
            torch.cuda.synchronize()
            assert torch.equal(single.lisi.view(torch.int32), res.lisi.view(torch.int32)), k
            assert torch.equal(single.auglisi.view(torch.int32), res.auglisi.view(torch.int32)), k
