"""The ragged-batch and serving workloads at their full sizes, in the launch
configuration the benchmark times.

* Ragged batch: 256 pairs, N drawn from {512, 1024, 2048, 4096} and N_T from
  {32, 64, 128}, in one persistent launch with the default wave count.  As in
  the benchmark, one generated pair per (N, transient or not) is copied into
  distinct device buffers for every pair.  Every tile of every pair is checked
  against the FP64 oracle, and every pair is bitwise equal to its single-pair
  launch with the batch geometry.
* Serving: 16 resident references with N round-robin over {1024, 2048, 4096},
  three distinct snapshots each, N_T from {32, 64}, Poisson arrivals at 20k
  requests/s.  Every result is bitwise equal to the single-pair launch of its
  own snapshot with the server's geometry, and one request per (reference,
  N_T) is checked against the oracle on every tile.
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import iqa_tiles, synth
from paper_2501_10653_amd.batch import Batch, batch_cfg
from paper_2501_10653_amd.serve import Server, serve_cfg
from tests.gpu_util import assert_parity, oracle_for, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_ragged_batch_full_config():
    specs = synth.ragged_specs(count=256, seed=7)
    print(f"ragged batch: {len(specs)} pairs", flush=True)
    host, proto = {}, {}
    for N in sorted({sp.N for sp in specs}):
        for kind in (0, 1):
            sp = synth.PairSpec(N=N, NT=64, n_src=synth.scaled_count(33, N, 1), amp_lo=1e-3,
                                amp_hi=2.0, fwhm=4.0, noise_sigma=1e-4,
                                n_drop=3 if kind else 0, seed=N * 10 + kind)
            x, y, _ = synth.make_pair(sp)
            host[(N, kind)] = (x, y)
            proto[(N, kind)] = (to_dev(x), to_dev(y))
    keys = [(sp.N, 1 if sp.n_drop else 0) for sp in specs]
    pairs = [(proto[k][0].clone(), proto[k][1].clone(), sp.NT) for k, sp in zip(keys, specs)]
    del proto
    b = Batch(pairs)
    assert b.count == len(pairs) and not b.single
    b.run()
    torch.cuda.synchronize()

    oracles = {}
    for i, (k, sp) in enumerate(zip(keys, specs)):
        key = (k, sp.NT)
        if key not in oracles:
            oracles[key] = oracle_for(host[k][0], host[k][1], sp.NT)
        assert_parity(b.results[i], oracles[key], what=f"pair {i} N={sp.N} NT={sp.NT}")
    for i, ((x, y, NT), sp) in enumerate(zip(pairs, specs)):
        single = iqa_tiles(x, y, NT, cfg=batch_cfg(sp.N, NT))
        torch.cuda.synchronize()
        assert same(single.lisi, b.results[i].lisi), f"pair {i}"
        assert same(single.auglisi, b.results[i].auglisi), f"pair {i}"


def test_serving_full_config():
    """400 requests over 16 references with three distinct snapshots each: a
    request that read another request's snapshot (or reference) would differ
    from its own single-pair launch."""
    specs = synth.serving_references(count=16, seed=11)
    print(f"serving: {len(specs)} references x 3 snapshots", flush=True)
    refs, snaps = [], []
    for sp in specs:
        x, _, _ = synth.make_pair(sp)
        refs.append((x, to_dev(x)))
        snaps.append([(s, to_dev(s)) for s in (synth.make_snapshot(sp, k) for k in range(3))])
    rng = np.random.default_rng(21)
    plan = [(int(rng.integers(len(specs))), int(rng.integers(3)), int(rng.choice([32, 64])))
            for _ in range(400)]
    with Server(16 << 30, streams=2, max_batch=512) as srv:
        ids = [srv.add_reference(d) for _, d in refs]
        reqs = [srv.request(snaps[r][k][1], ids[r], NT) for r, k, NT in plan]
        arrivals = synth.poisson_arrivals(20000.0, len(reqs), seed=4)
        comps = srv.replay(reqs, arrivals, timeout_s=120.0)
        st = srv.stats()
    assert len(comps) == len(reqs) and all(c["status"] == 0 for c in comps)
    assert st["completed"] == len(reqs) and st["rejected"] == 0

    singles = {}
    for (r, k, NT), req in zip(plan, reqs):
        if (r, k, NT) not in singles:
            N = specs[r].N
            singles[(r, k, NT)] = iqa_tiles(snaps[r][k][1], refs[r][1], NT, cfg=serve_cfg(N, NT))
            torch.cuda.synchronize()
        one = singles[(r, k, NT)]
        assert same(one.lisi, req.lisi) and same(one.auglisi, req.auglisi), (r, k, NT)
    # the snapshots of one reference differ, so their results do too
    for r in range(len(specs)):
        got = [singles.get((r, k, 64)) for k in range(3)]
        got = [g for g in got if g is not None]
        for a, b in zip(got, got[1:]):
            assert not same(a.auglisi, b.auglisi), r
    # every (reference, N_T) against the oracle on one of its snapshots
    seen = set()
    for (r, k, NT), one in singles.items():
        if (r, NT) in seen:
            continue
        seen.add((r, NT))
        assert_parity(one, oracle_for(snaps[r][k][0], refs[r][0], NT),
                      what=f"ref {r} snapshot {k} NT={NT}")


def test_serving_under_overload():
    """20,000 requests arriving at 100k/s, beyond what the device can serve:
    batches grow past the inline limit (device descriptor table), slots are
    reused as fast as their completion words arrive, and every result still
    equals its single-pair launch bitwise.  N_T 128 is mixed in, so pairs of
    one- and four-wave geometries share batches."""
    specs = synth.serving_references(count=16, seed=11)
    refs, snaps = [], []
    for sp in specs:
        x, _, _ = synth.make_pair(sp)
        refs.append(to_dev(x))
        snaps.append(to_dev(synth.make_snapshot(sp, 1)))
    rng = np.random.default_rng(23)
    plan = [(int(rng.integers(len(specs))), int(rng.choice([32, 64, 128]))) for _ in range(20000)]
    print(f"overload: {len(plan)} requests at 100k/s", flush=True)
    with Server(32 << 30, streams=4, max_batch=512) as srv:
        ids = [srv.add_reference(d) for d in refs]
        reqs = [srv.request(snaps[r], ids[r], NT) for r, NT in plan]
        arrivals = synth.poisson_arrivals(100000.0, len(reqs), seed=5)
        comps = srv.replay(reqs, arrivals, timeout_s=120.0)
        st = srv.stats()
    assert len(comps) == len(reqs) and all(c["status"] == 0 for c in comps)
    assert st["completed"] == len(reqs) and st["max_batch"] > 16
    singles = {}
    for (r, NT), req in zip(plan, reqs):
        if (r, NT) not in singles:
            singles[(r, NT)] = iqa_tiles(snaps[r], refs[r], NT, cfg=serve_cfg(specs[r].N, NT))
            torch.cuda.synchronize()
        one = singles[(r, NT)]
        assert same(one.lisi, req.lisi) and same(one.auglisi, req.auglisi), (r, NT)
