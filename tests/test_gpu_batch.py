"""Ragged batches in one persistent launch: every pair bitwise equal to its
single-pair launch with the same geometry, and within tolerance of the oracle;
graph replays equal the eager run."""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import iqa_tiles, synth
from paper_2501_10653_amd.batch import Batch, batch_cfg
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

# N_T 512 and 1024 take the kernel's wide path (a tile row wider than one
# 64-lane segment); the rest the narrow one.
SHAPES = [(64, 16), (128, 32), (256, 64), (512, 128), (1024, 32), (1024, 64), (512, 256),
          (2048, 128), (96, 48), (300, 12), (1000, 20), (768, 256), (128, 128), (4096, 64),
          (1024, 512), (2048, 1024)]


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.fixture(scope="module")
def ragged():
    rng = np.random.default_rng(77)
    host, dev = [], []
    order = list(SHAPES) * 2
    rng.shuffle(order)
    for N, NT in order:
        x, y = synth.random_pair(N, rng, neg_frac=0.3, nan_frac=0.01, scale=1.5)
        host.append((x, y, NT))
        dev.append((to_dev(x), to_dev(y), NT))
    return host, dev


def test_batch_matches_single_launches_bitwise(ragged):
    host, dev = ragged
    b = Batch(dev, sums=True)
    b.run()
    torch.cuda.synchronize()
    for (xd, yd, NT), res in zip(dev, b.results):
        N = xd.shape[0]
        single = iqa_tiles(xd, yd, NT, sums=True, cfg=batch_cfg(N, NT))
        torch.cuda.synchronize()
        assert same(res.lisi, single.lisi) and same(res.auglisi, single.auglisi)
        assert same(res.sums, single.sums)


def test_batch_parity_with_oracle(ragged):
    host, dev = ragged
    b = Batch(dev, sums=True)
    b.run()
    torch.cuda.synchronize()
    for (x, y, NT), res in zip(host, b.results):
        assert_parity(res, oracle_for(x, y, NT), what=f"{x.shape[0]}/{NT}")


@pytest.mark.parametrize("waves", [4, 64, 1024, 4096])
def test_wave_count_does_not_change_bits(ragged, waves):
    _, dev = ragged
    ref = Batch(dev)
    ref.run()
    b = Batch(dev, waves=waves)
    b.run()
    torch.cuda.synchronize()
    for r0, r1 in zip(ref.results, b.results):
        assert same(r0.lisi, r1.lisi) and same(r0.auglisi, r1.auglisi)


def test_graph_replays_equal_eager(ragged):
    _, dev = ragged
    b = Batch(dev)
    s = torch.cuda.Stream()
    b.run(stream=s)
    torch.cuda.synchronize()
    eager = [(r.lisi.clone(), r.auglisi.clone()) for r in b.results]
    g = b.capture(s)
    for rep in range(3):
        for r in b.results:
            r.lisi.fill_(-1.0)
            r.auglisi.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        for (l0, a0), r in zip(eager, b.results):
            assert same(l0, r.lisi) and same(a0, r.auglisi), rep


def test_inline_descriptors_equal_device_table(ragged):
    """Up to IQA_BATCH_INLINE_MAX pairs with their descriptors in the kernel
    arguments: bitwise the launch from a device table, eager and replayed."""
    host, dev = ragged
    sub = [p for p in dev if p[2] % 4 == 0][:16]
    assert len(sub) == 16
    table = Batch(sub, sums=True, inline=False)
    inl = Batch(sub, sums=True)
    assert inl.inline and inl.descs is None and not table.inline
    s = torch.cuda.Stream()
    table.run(stream=s)
    inl.run(stream=s)
    torch.cuda.synchronize()
    for r0, r1 in zip(table.results, inl.results):
        assert same(r0.lisi, r1.lisi) and same(r0.auglisi, r1.auglisi) and same(r0.sums, r1.sums)
    eager = [(r.lisi.clone(), r.auglisi.clone()) for r in inl.results]
    g = inl.capture(s)
    for rep in range(3):
        for r in inl.results:
            r.lisi.fill_(-1.0)
            r.auglisi.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        for (l0, a0), r in zip(eager, inl.results):
            assert same(l0, r.lisi) and same(a0, r.auglisi), rep
    with pytest.raises(ValueError):
        Batch(dev[:17] if len(dev) >= 17 else dev * 2, inline=True)


@pytest.mark.parametrize("k", [1, 2, 4, 5, 15])
def test_inline_argument_sizes_equal_device_table(ragged, k):
    """Batches of 1..16 pairs launch with an argument block of 1, 4 or 16
    descriptors; every size gives the device-table launch's bits."""
    host, dev = ragged
    sub = [p for p in dev if p[2] % 4 == 0][:k]
    table = Batch(sub, sums=True, inline=False)
    inl = Batch(sub, sums=True)
    assert inl.inline
    table.run()
    inl.run()
    torch.cuda.synchronize()
    for r0, r1 in zip(table.results, inl.results):
        assert same(r0.lisi, r1.lisi) and same(r0.auglisi, r1.auglisi) and same(r0.sums, r1.sums)


@pytest.mark.parametrize("rp", [1, 2, 4])
def test_four_wave_geometry_matches_single_launch_and_oracle(ragged, rp):
    """Pairs whose batch geometry has the four waves of a workgroup split each
    tile group's rows: bitwise the single-pair launch with that geometry, and
    within tolerance of the oracle, mixed in one batch with one-wave pairs."""
    from paper_2501_10653_amd import _lib
    from paper_2501_10653_amd._lib import LaunchCfg
    host, dev = ragged
    lib = _lib.load()
    coop = set()
    try:
        for (x, y, NT) in host:
            N = x.shape[0]
            if NT % 4 or (N, NT) in coop or len(coop) >= 6:
                continue
            lpt = NT // 4
            seg = min(64, 1 << (lpt - 1).bit_length())
            if seg * rp > 64 or NT % 4:
                continue
            cfg = dict(vec=4, waves=4, unroll=8, seg=seg, rp=rp, ksplit=1)
            assert lib.iqa_tune_set(N, NT, _lib.TUNE_BATCH, LaunchCfg.from_dict(cfg)) == 0
            coop.add((N, NT))
        assert coop
        b = Batch(dev, sums=True)
        b.run()
        torch.cuda.synchronize()
        for (x, y, NT), (xd, yd, _), res in zip(host, dev, b.results):
            N = x.shape[0]
            if (N, NT) in coop:
                assert batch_cfg(N, NT)["waves"] == 4
            single = iqa_tiles(xd, yd, NT, sums=True, cfg=batch_cfg(N, NT))
            torch.cuda.synchronize()
            assert same(res.lisi, single.lisi) and same(res.auglisi, single.auglisi), (N, NT)
            assert same(res.sums, single.sums), (N, NT)
            assert_parity(res, oracle_for(x, y, NT), what=f"{N}/{NT} rp {rp}")
    finally:
        lib.iqa_tune_clear()


def test_units_outside_the_table_are_skipped(ragged):
    """A table launch told of more units than described, and of fewer pairs
    than the table holds: the units past the pairs it was given are skipped.
    The pairs launched come out bitwise as in the full batch; the others keep
    what their outputs held."""
    import ctypes
    from paper_2501_10653_amd import _lib
    host, dev = ragged
    sub = [p for p in dev if p[2] % 4 == 0][:6]
    full = Batch(sub, inline=False)
    full.run()
    part = Batch(sub, inline=False)
    for r in part.results:
        r.lisi.fill_(-1.0)
        r.auglisi.fill_(-1.0)
    torch.cuda.synchronize()
    k = 4
    st = _lib.load().iqa_tiles_batched(part.descs.data_ptr(), k, part.units + 1000, part.waves,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    for i, (r0, r1) in enumerate(zip(full.results, part.results)):
        if i < k:
            assert same(r0.lisi, r1.lisi) and same(r0.auglisi, r1.auglisi), i
        else:
            assert bool((r1.lisi == -1.0).all()) and bool((r1.auglisi == -1.0).all()), i


def test_paper_recipe_pairs_in_a_batch():
    """Pairs built like the ragged-batch workload (sources removed in some,
    noise-only changes in the others) at mixed sizes up to 4096."""
    specs = synth.ragged_specs(count=6, seed=3)
    host, dev = [], []
    for sp in specs:
        x, y, _ = synth.make_pair(sp)
        host.append((x, y, sp.NT))
        dev.append((to_dev(x), to_dev(y), sp.NT))
    b = Batch(dev)
    b.run()
    torch.cuda.synchronize()
    for (x, y, NT), res in zip(host, b.results):
        assert_parity(res, oracle_for(x, y, NT), what=f"{x.shape[0]}/{NT}")


def test_batch_with_pairs_the_persistent_kernel_cannot_take():
    """N_T not a multiple of 4, and an image 4 bytes off a 16-byte boundary,
    are launched singly inside Batch.run; every result matches the oracle."""
    rng = np.random.default_rng(31)
    host, dev = [], []
    for N, NT, off in [(300, 12, 0), (90, 6, 0), (81, 9, 0), (256, 32, 1), (512, 64, 0)]:
        x, y = synth.random_pair(N, rng, neg_frac=0.3, scale=1.0)
        xd = torch.zeros(N * N + 4, device="cuda")[off:off + N * N].view(N, N)
        xd.copy_(to_dev(x))
        host.append((x, y, NT))
        dev.append((xd, to_dev(y), NT))
    b = Batch(dev, sums=True)
    assert sorted(b.single) == [1, 2, 3]
    b.run()
    torch.cuda.synchronize()
    for (x, y, NT), res in zip(host, b.results):
        assert_parity(res, oracle_for(x, y, NT), what=f"{x.shape[0]}/{NT}")
