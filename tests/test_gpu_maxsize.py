"""Maximum sizes: the largest image side the ABI accepts (2^17, a 128 GiB
pair) and a 2^16 image with small tiles, checked on sampled tiles that the
oracle recomputes one by one from their pixels."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2501_10653_amd import iqa_tiles
from tests.gpu_util import assert_parity, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.mark.parametrize("N,NT", [(1 << 17, 1024), (1 << 16, 64)])
def test_maximum_sizes_sampled(N, NT):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 8 * N * N * 1.05:
        pytest.skip(f"needs {8 * N * N / 2**30:.0f} GiB of free device memory")
    g = torch.Generator(device="cuda")
    g.manual_seed(N + NT)
    x = torch.empty(N, N, device="cuda").uniform_(-0.3, 1.0, generator=g)
    y = torch.empty(N, N, device="cuda").uniform_(-0.3, 1.0, generator=g)
    try:
        res = iqa_tiles(x, y, NT, sums=True)
        torch.cuda.synchronize()
        ns = N // NT
        rng = np.random.default_rng(N)
        picks = [(0, 0), (0, ns - 1), (ns - 1, 0), (ns - 1, ns - 1)] + \
            [tuple(int(v) for v in rng.integers(0, ns, 2)) for _ in range(12)]
        c = oracle.f32const(1e-6)
        for ty, tx in picks:
            xb = x[ty * NT:(ty + 1) * NT, tx * NT:(tx + 1) * NT].cpu().numpy()
            yb = y[ty * NT:(ty + 1) * NT, tx * NT:(tx + 1) * NT].cpu().numpy()
            ol, oa, os_ = oracle.iqa_tiles(xb, yb, NT, c / 2, c, c, c)
            t = ty * ns + tx

            class One:
                lisi = res.lisi[ty, tx].reshape(1, 1)
                auglisi = res.auglisi[ty, tx].reshape(1, 1)
                sums = res.sums[t].reshape(1, 4)
            assert_parity(One, (ol, oa, os_), what=f"{N}/{NT} tile ({ty},{tx})")
    finally:
        del x, y
        torch.cuda.empty_cache()
