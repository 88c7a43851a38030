"""Seeded random sweep over shapes, launch configurations, image offsets and
constants, every case against the oracle on every tile.

Each case draws an image side N <= 640 and a tile side dividing it, a launch
configuration that the library accepts for that shape (vector width, waves,
unroll, segment width, row phases, split factor), a pointer offset that
decides the alignment the vector width needs, and the four constants.  The
fixed seed makes the sweep the same on every run.
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import check_cfg, iqa_tiles, prepare, synth
from tests.gpu_util import assert_parity, oracle_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = 160


def _draw(rng):
    while True:
        NT = int(rng.choice([1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128, 256]))
        ns = int(rng.integers(1, max(2, 640 // NT) + 1))
        N = NT * ns
        if N > 640:
            continue
        vec = int(rng.choice([v for v in (1, 2, 4) if NT % v == 0]))
        lpt = NT // vec
        seg_full = min(64, 1 << (lpt - 1).bit_length())
        seg = int(rng.choice([s for s in (seg_full, seg_full // 2) if s >= 1]))
        rp = int(rng.choice([r for r in (1, 2, 4, 8) if seg * r <= 64]))
        waves = int(rng.choice([1, 2, 4, 8, 16] if vec == 4 else [1, 4]))
        unroll = int(rng.choice([4, 8] if vec == 4 and waves <= 8 else [4]))
        ks = int(rng.choice([1, 1, 2, 4]))
        cfg = dict(vec=vec, waves=waves, unroll=unroll, seg=seg, rp=rp, ksplit=ks)
        if check_cfg(N, NT, cfg) == 0:
            return N, NT, cfg


def _cases():
    rng = np.random.default_rng(2025)
    out = []
    for i in range(CASES):
        N, NT, cfg = _draw(rng)
        off = int(rng.choice([0, 0, cfg["vec"], 2 * cfg["vec"]]))    # floats; keeps vec alignment
        C1, C2, C = (float(v) for v in 10.0 ** rng.uniform(-7, -3, 3))
        D = float(10.0 ** rng.uniform(-7, -3))
        out.append((i, N, NT, cfg, off, C1, C2, C, D))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}/{c[2]}")
def test_random_case_against_oracle(case):
    i, N, NT, cfg, off, C1, C2, C, D = case
    rng = np.random.default_rng((7, i))
    x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01, scale=float(rng.uniform(0.1, 3)))
    dev = torch.device("cuda", 0)
    bx = torch.empty(N * N + off + 64, device=dev)
    by = torch.empty(N * N + off + 64, device=dev)
    xd = bx[off:off + N * N].view(N, N)
    yd = by[off:off + N * N].view(N, N)
    xd.copy_(torch.from_numpy(x))
    yd.copy_(torch.from_numpy(y))
    prepare(N, NT, cfg)
    res = iqa_tiles(xd, yd, NT, C1=C1, C2=C2, C=C, D=D, sums=True, cfg=cfg)
    torch.cuda.synchronize()
    assert_parity(res, oracle_for(x, y, NT, C1=C1, C2=C2, C=C, D=D),
                  what=f"case {i}: N={N} NT={NT} cfg={cfg} off={off}")
