"""iqa_tiles_noalloc, called through the C ABI: the same bits as iqa_tiles_cfg
with the same launch configuration on split shapes (whose partial sums live
in the library's fixed scratch array) and on a shape that does not split, on
calls in a row with a smaller input second.  (Shapes needing more scratch
than the array holds are refused before any HIP call: a CPU test.)"""

from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import _lib, default_cfg, synth
from paper_2501_10653_amd._lib import LaunchCfg
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

C6 = 1e-6
D6 = float(np.float32(C6)) / 2.0


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def call(fn, xd, yd, NT, cfg, stream):
    """One C-ABI call of `fn` (iqa_tiles_cfg or iqa_tiles_noalloc) with fresh
    outputs; returns (status, lisi, auglisi, sums)."""
    N = xd.shape[0]
    ns = N // NT
    lo = torch.full((ns, ns), -1.0, device="cuda")
    ao = torch.full((ns, ns), -1.0, device="cuda")
    so = torch.full((ns * ns, 4), -1.0, device="cuda")
    torch.cuda.synchronize()
    st = fn(xd.data_ptr(), yd.data_ptr(), N, NT, D6, C6, C6, C6, lo.data_ptr(), ao.data_ptr(),
            so.data_ptr(), ctypes.byref(LaunchCfg.from_dict(cfg)), stream.cuda_stream)
    torch.cuda.synchronize()
    return st, lo, ao, so


@pytest.mark.parametrize("shapes", [
    [(2048, 256, None), (1024, 256, None)],      # default split shapes, second smaller
    [(1024, 512, 32), (512, 512, 8)],            # deep split, then a shallower smaller one
    [(2048, 64, None), (256, 32, None)],         # no split: no scratch used
    [(2048, 128, 8), (1024, 128, 8)],            # one wave per workgroup: combine launches
])
def test_noalloc_equals_allocating_entry_point(shapes):
    lib = _lib.load()
    s = torch.cuda.Stream()
    rng = np.random.default_rng(sum(N + NT for N, NT, _ in shapes))
    for N, NT, ks in shapes:
        x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01, scale=1.0)
        xd, yd = to_dev(x), to_dev(y)
        cfg = default_cfg(N, NT, xd, yd)
        if ks is not None:
            cfg["ksplit"] = ks
            if NT == 128 and ks == 8:
                cfg.update(waves=1, unroll=8)
        print(f"noalloc N={N} NT={NT} cfg={cfg}", flush=True)
        st0, l0, a0, s0 = call(lib.iqa_tiles_cfg, xd, yd, NT, cfg, s)
        st1, l1, a1, s1 = call(lib.iqa_tiles_noalloc, xd, yd, NT, cfg, s)
        assert st0 == 0 and st1 == 0, (st0, st1)
        assert same(l0, l1) and same(a0, a1) and same(s0, s1), (N, NT, cfg)
        from paper_2501_10653_amd.iqa import TileResult
        assert_parity(TileResult(l1, a1, s1), oracle_for(x, y, NT), what=f"{N}/{NT} {cfg}")


def test_noalloc_repeated_calls_on_one_stream():
    """Split launches back to back on one stream through the scratch array:
    each leaves its ticket counters at zero for the next."""
    lib = _lib.load()
    s = torch.cuda.Stream()
    rng = np.random.default_rng(8)
    N, NT = 1024, 256
    x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
    xd, yd = to_dev(x), to_dev(y)
    cfg = default_cfg(N, NT, xd, yd)
    assert cfg["ksplit"] > 1
    st, l0, a0, _ = call(lib.iqa_tiles_cfg, xd, yd, NT, cfg, s)
    assert st == 0
    ns = N // NT
    outs = [(torch.empty(ns, ns, device="cuda"), torch.empty(ns, ns, device="cuda"))
            for _ in range(50)]
    for lo, ao in outs:
        st = lib.iqa_tiles_noalloc(xd.data_ptr(), yd.data_ptr(), N, NT, D6, C6, C6, C6,
                                   lo.data_ptr(), ao.data_ptr(), None,
                                   ctypes.byref(LaunchCfg.from_dict(cfg)), s.cuda_stream)
        assert st == 0
    torch.cuda.synchronize()
    for lo, ao in outs:
        assert same(lo, l0) and same(ao, a0)
