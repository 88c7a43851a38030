"""Autotuner for the launch shapes of the tile kernels.

For a single image pair of shape (N, N_T) it times every valid candidate
launch configuration (waves per workgroup, rows per load batch, row phases per
wave, workgroups per tile) and keeps the fastest.  For ragged batches it
picks, per N_T, the per-pair geometry (row phases per wave) and the number of
persistent waves.  Timing replays a HIP graph of K launches that rotate over a
pool of distinct device copies of the pair (more bytes than the 256 MB
Infinity Cache), so every launch streams from HBM.

Results go to a JSON cache (``tuned/gfx950.json`` next to this file), which
the build embeds into the library as its default shapes.

    python -m paper_2501_10653_amd.tune --sweep --batch --out paper_2501_10653_amd/tuned/gfx950.json
"""

from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuned", "gfx950.json")

SWEEP = [(N, NT) for N in (1024, 2048, 4096, 8192) for NT in (16, 32, 64, 128, 256)]
EXTRA = [(256, 32), (512, 32), (512, 64), (512, 128), (1024, 512), (2048, 512), (4096, 512)]


def candidates_single(N: int, NT: int, max_waves_total: int = 1 << 17) -> List[dict]:
    """Valid vec-4 configurations worth timing for (N, NT)."""
    from .iqa import check_cfg
    if NT % 4:
        return []
    lpt = NT // 4
    seg = min(64, 1 << (lpt - 1).bit_length())
    tpw = 64 // seg
    ns = N // NT
    out = []
    combos = [(w, u) for w in (1, 2, 4, 8) for u in (4, 8)] + [(16, 4)]
    for (waves, unroll), rp_log, ks_log in itertools.product(combos, range(7), range(10)):
        rp, ks = 1 << rp_log, 1 << ks_log
        if rp > tpw:
            continue
        cfg = dict(vec=4, waves=waves, unroll=unroll, seg=seg, rp=rp, ksplit=ks)
        if check_cfg(N, NT, cfg) != 0:
            continue
        ht = tpw // rp
        total = ns * math.ceil(ns / ht) * ks * waves
        rows_per_lane = NT / (rp * waves * ks)
        if total < 128 or total > max_waves_total or rows_per_lane < 2:
            continue
        out.append(cfg)
    return out


class _Timer:
    """Graph-replay timing on one stream with a rotating pool of pairs: the
    measurement harness's rule (K launches in one graph, an untimed replay,
    then timed replays each behind a read-only prelude)."""

    def __init__(self, torch, stream):
        from .measure import GraphTimer
        self.timer = GraphTimer(torch, torch.device("cuda", torch.cuda.current_device()), stream)

    def per_launch_us(self, launch, K: int, reps: int = 5) -> float:
        return self.timer.per_launch_us(launch, K, reps=reps)


def evict_infinity_cache(torch, dev, nbytes: int = 512 << 20, passes: int = 4) -> None:
    """Age out whatever the 256 MB Infinity Cache holds before a timing:
    several passes of ordinary loads over a scratch buffer twice its size."""
    buf = torch.ones(nbytes // 4, device=dev)
    for _ in range(passes):
        float(buf.sum())
    del buf


def device_copies(torch, dev, arr, count: int):
    """`count` distinct device copies of a host array, each uploaded from the
    host, so that no copy has been read on the device before a timing."""
    host = torch.from_numpy(arr)
    return [host.to(dev) for _ in range(count)]


def _pool(torch, dev, N: int, NT: int, pool_bytes: float):
    from . import synth
    x, y, _ = synth.make_pair(synth.spec_sweep(N, NT))
    n = max(2, int(math.ceil(pool_bytes / (8 * N * N))))
    xs = device_copies(torch, dev, x, n)
    ys = device_copies(torch, dev, y, n)
    evict_infinity_cache(torch, dev)
    return xs, ys


def tune_single(N: int, NT: int, pool_bytes: float = 2 ** 30, K: int = 64,
                log=None, refine: int = 3,
                rounds: int = 3) -> Tuple[dict, float, List[Tuple[float, dict]]]:
    """Time every candidate for (N, NT), then re-time the `refine` fastest
    with longer graphs; returns (best cfg, best us, all, best first)."""
    import torch
    from .iqa import default_cfg, iqa_tiles, prepare
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(dev)
    xs, ys = _pool(torch, dev, N, NT, pool_bytes)
    ns = N // NT
    out = {"lisi": torch.empty(ns, ns, device=dev), "auglisi": torch.empty(ns, ns, device=dev)}
    timer = _Timer(torch, s)
    pool = len(xs)
    K = max(K, pool)
    results = []
    cands = candidates_single(N, NT)
    base = default_cfg(N, NT)
    if base not in cands:
        cands.append(base)
    for cfg in cands:
        prepare(N, NT, cfg, stream=s)
        us = timer.per_launch_us(
            lambda i: iqa_tiles(xs[i % pool], ys[i % pool], NT, out=out, cfg=cfg, stream=s), K)
        results.append((us, cfg))
        if log:
            log(f"  {N}/{NT} {us:8.2f} us {cfg}")
    results.sort(key=lambda r: r[0])
    # The leaders are often within the noise of one short replay: time the
    # top few again with longer graphs, in interleaved rounds, and rank them
    # by the median over the rounds.
    top = results[:refine]
    if len(top) > 1:
        K2 = max(4 * K, 256)
        runs = {i: [] for i in range(len(top))}
        for _ in range(rounds):
            for i, (_, cfg) in enumerate(top):
                runs[i].append(timer.per_launch_us(
                    lambda j: iqa_tiles(xs[j % pool], ys[j % pool], NT, out=out, cfg=cfg,
                                        stream=s), K2, reps=3))
        top = sorted(((float(np.median(runs[i])), cfg) for i, (_, cfg) in enumerate(top)),
                     key=lambda r: r[0])
        if log:
            for us, cfg in top:
                log(f"  {N}/{NT} refined {us:8.3f} us {cfg}")
        results = top + results[len(top):]
    del xs, ys
    torch.cuda.empty_cache()
    return results[0][1], results[0][0], results


def candidates_batch(NT: int) -> List[dict]:
    """Per-pair batch geometries: one wave per tile group (waves 1) or the
    four waves of a workgroup splitting each tile group's rows (waves 4), at
    every row-phase count a wave allows."""
    lpt = NT // 4
    seg = min(64, 1 << (lpt - 1).bit_length())
    tpw = 64 // seg
    return [dict(vec=4, waves=w, unroll=8, seg=seg, rp=1 << r, ksplit=1)
            for w in (1, 4) for r in range(7) if (1 << r) <= tpw]


def tune_batch(NTs: Sequence[int] = (32, 64, 128), Ns: Sequence[int] = (512, 1024, 2048, 4096),
               copies: int = 8, waves_list: Sequence[int] = (1024, 2048, 4096, 8192, 16384),
               log=None) -> Tuple[Dict[int, dict], int, list]:
    """Per-N_T batch geometry and the persistent wave count, timed on a batch
    of `copies` pairs of every (N, N_T)."""
    import torch
    from . import _lib, synth
    from ._lib import LaunchCfg
    from .batch import Batch
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(dev)
    timer = _Timer(torch, s)
    proto = {}
    for N in Ns:
        x, y, _ = synth.make_pair(synth.spec_sweep(N, 64))
        proto[N] = (torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    lib = _lib.load()
    best: Dict[int, dict] = {}
    log_rows = []
    for NT in NTs:
        pairs = [(proto[N][0].clone(), proto[N][1].clone(), NT) for N in Ns for _ in range(copies)]
        evict_infinity_cache(torch, dev)
        total = sum(8 * p[0].shape[0] ** 2 for p in pairs)
        res = []
        for cfg in candidates_batch(NT):
            for N in Ns:
                _lib.check(lib.iqa_tune_set(N, NT, _lib.TUNE_BATCH,
                                            LaunchCfg.from_dict(cfg)), "iqa_tune_set")
            b = Batch(pairs, waves=2048)
            us = timer.per_launch_us(lambda i: b.run(stream=s), 4)
            res.append((us, cfg))
            log_rows.append({"NT": NT, "cfg": cfg, "us": us, "gbs": total / us / 1e3})
            if log:
                log(f"  batch NT={NT} {us:9.1f} us {total / us / 1e3:7.0f} GB/s {cfg}")
        res.sort(key=lambda r: r[0])
        best[NT] = res[0][1]
        for N in Ns:
            lib.iqa_tune_set(N, NT, _lib.TUNE_BATCH, LaunchCfg.from_dict(best[NT]))
        del pairs
    # Persistent waves, scored on two batches: a large mixed one (every N and
    # N_T) and a small one (three pairs, as a server sees at moderate load),
    # where too few waves leave a second round of units for some of them.
    mixed = [(proto[N][0].clone(), proto[N][1].clone(), NT) for N in Ns for NT in NTs
             for _ in range(max(1, copies // 2))]
    smalls = [[(proto[N][0].clone(), proto[N][1].clone(), NT)
               for N, NT in zip(Ns[-3:], (32, 64, 64))] for _ in range(8)]
    evict_infinity_cache(torch, dev)
    total = sum(8 * p[0].shape[0] ** 2 for p in mixed)
    t_mixed, t_small = {}, {}
    for w in waves_list:
        b = Batch(mixed, waves=w)
        t_mixed[w] = timer.per_launch_us(lambda i: b.run(stream=s), 4)
        bs = [Batch(p, waves=w) for p in smalls]
        t_small[w] = timer.per_launch_us(lambda i: bs[i % len(bs)].run(stream=s), 32)
        log_rows.append({"NT": "mixed", "waves": w, "us": t_mixed[w],
                         "gbs": total / t_mixed[w] / 1e3, "small_batch_us": t_small[w]})
        if log:
            log(f"  batch waves={w} mixed {t_mixed[w]:9.1f} us {total / t_mixed[w] / 1e3:7.0f} GB/s"
                f"  small {t_small[w]:7.2f} us")
    m0, s0 = min(t_mixed.values()), min(t_small.values())
    best_w = min(waves_list, key=lambda w: t_mixed[w] / m0 + t_small[w] / s0)
    lib.iqa_tune_clear()
    return best, best_w, log_rows


SERVE_SHAPES = [(N, NT) for N in (512, 1024, 2048, 4096) for NT in (32, 64, 128)]


def tune_serve(shapes: Sequence[Tuple[int, int]] = tuple(SERVE_SHAPES), K: int = 64,
               refine: int = 3, rounds: int = 3, log=None) -> Tuple[Dict[str, dict], list]:
    """Per-(N, N_T) geometry for the server's batches, chosen for latency:
    the time of a batch that holds one pair (as a server's batches mostly
    do), in graph replays over distinct copies; the fastest few are then
    re-timed in longer graphs over interleaved rounds."""
    import torch
    from . import _lib, synth
    from ._lib import LaunchCfg
    from .batch import Batch
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(dev)
    timer = _Timer(torch, s)
    lib = _lib.load()
    best: Dict[str, dict] = {}
    log_rows = []
    for N in sorted({N for N, _ in shapes}):
        x, y, _ = synth.make_pair(synth.spec_sweep(N, 64))
        n = max(4, min(64, int(math.ceil((1 << 30) / (8 * N * N)))))
        xs = device_copies(torch, dev, x, n)
        ys = device_copies(torch, dev, y, n)
        for NT in sorted({nt for n2, nt in shapes if n2 == N}):
            def timed(cfg, K):
                # the geometry is timed through the batch table; only the
                # geometry matters to the kernel, not which table holds it
                _lib.check(lib.iqa_tune_set(N, NT, _lib.TUNE_BATCH, LaunchCfg.from_dict(cfg)),
                           "iqa_tune_set")
                bs = [Batch([(xs[i], ys[i], NT)]) for i in range(n)]
                evict_infinity_cache(torch, dev)
                us = timer.per_launch_us(lambda i: bs[i % n].run(stream=s), K)
                lib.iqa_tune_clear()
                return us
            res = sorted((timed(c, K), i, c) for i, c in enumerate(candidates_batch(NT)))
            top = [c for _, _, c in res[:refine]]
            again = {i: [] for i in range(len(top))}
            for _ in range(rounds):
                for i, c in enumerate(top):
                    again[i].append(timed(c, 4 * K))
            med = sorted((float(np.median(again[i])), i) for i in range(len(top)))
            us, i = med[0]
            best[f"{N}x{NT}"] = top[i]
            log_rows.append({"N": N, "NT": NT, "cfg": top[i], "us": round(us, 3),
                             "first_pass": [{"cfg": c, "us": round(u, 3)} for u, _, c in res]})
            if log:
                log(f"  serve {N}/{NT}: {us:.2f} us {top[i]}")
        del xs, ys
    return best, log_rows


def load(path: str = DEFAULT_OUT) -> Optional[dict]:
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--shapes", default="", help="comma list of N:NT")
    ap.add_argument("--sweep", action="store_true", help="the N x N_T size-sweep grid")
    ap.add_argument("--batch", action="store_true", help="tune ragged-batch geometry")
    ap.add_argument("--serve", action="store_true", help="tune the server's (lone-pair) geometry")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--K", type=int, default=64)
    args = ap.parse_args(argv)
    import torch

    shapes = []
    if args.sweep:
        shapes += SWEEP + EXTRA
    for item in filter(None, args.shapes.split(",")):
        N, NT = (int(v) for v in item.split(":"))
        shapes.append((N, NT))
    doc = load(args.out) or {}
    doc.setdefault("arch", torch.cuda.get_device_properties(0).gcnArchName.split(":")[0])
    doc.setdefault("single", {})
    t0 = time.time()

    def log(msg):
        print(msg, flush=True)

    for N, NT in shapes:
        cfg, us, res = tune_single(N, NT, K=args.K, log=log)
        doc["single"][f"{N}x{NT}"] = {"cfg": cfg, "us": round(us, 3),
                                      "gbs": round(8 * N * N / us / 1e3, 1),
                                      "runner_up": [{"cfg": c, "us": round(u, 3)}
                                                    for u, c in res[1:4]]}
        log(f"{N}/{NT}: best {us:.2f} us ({8 * N * N / us / 1e3:.0f} GB/s) {cfg}")
    if args.batch:
        best, waves, rows = tune_batch(log=log)
        doc["batch"] = {str(NT): cfg for NT, cfg in best.items()}
        doc["batch_waves"] = waves
        doc["batch_log"] = rows
    if args.serve:
        best, rows = tune_serve(log=log)
        doc["serve"] = best
        doc["serve_log"] = rows
    doc["tuned_at_s"] = round(time.time() - t0, 1)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    log(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
