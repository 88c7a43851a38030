#!/usr/bin/env python3
"""Benchmark of the fused tile-wise LISI + augLISI path on one MI355X.

A step is one fused launch (clamp, per-pixel terms, per-tile compensated
reduction, Eq. 1 and Eq. 2 finalisation) over one synthetic FP32 image pair of
the paper's shape: N = 2048, N_T = 64 (32 x 32 IQA matrix).  Inputs are
resident in HBM before the timed region.  Steps rotate over a pool of distinct
device copies of the pair (>= 1 GiB in total) so that no step is served from
the 256 MB Infinity Cache that the previous steps filled.  The K timed steps
are K launches queued behind a prelude of plain reads on the stream (eager
launches up to 64 steps, one replay of a HIP graph holding exactly K launches
above): the timed region starts with the K launches already queued, so it
measures the GPU's back-to-back rate, not the host's submission delay.

The default run also reports, on the same GPU: the fastest plain read of the
same bytes, the 2 GiB read ceiling, the paper's two separate kernels, a
same-shape batch, the 256-pair ragged batch (one persistent launch in a graph
against 256 single-pair launches), serving at 2k, 10k and 50k requests/s
(throughput, p50 and p99 latency to the caller's poll) and the FP64 oracle on
the host cores (median of 10 runs per configuration, one thread and all).

Other workloads: ``--workload readfloor`` (plain reads and empty launches of
the pair's byte count in many shapes), ``timeline`` (per-workgroup timeline of
the fused launch), ``sweep`` (every cell of the size sweep), ``ragged``,
``serve``.  ``--plan-out`` writes the launch plan that
``python -m paper_2501_10653_amd.measure`` matches against a rocprofv3 trace.

Prints one JSON line.  ``--gpus N`` with N > 1 is not supported: this is a
single-GPU path.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from typing import Optional

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fused LISI+augLISI HBM GB/s (% peak) at 2048²/NT64; p99 request latency"
HBM_PEAK_GBS = 8000.0       # MI355X published HBM3E bandwidth
KERNEL_SRC = os.path.join(ROOT, "paper_2501_10653_amd", "csrc", "iqa_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
SWEEP_CELLS = [(N, NT) for N in (1024, 2048, 4096, 8192) for NT in (16, 32, 64, 128, 256)]
EAGER_MAX_STEPS = 64        # --graph auto: eager launches up to this many steps


def log(msg: str) -> None:
    """Progress of the run, on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="paper",
                    help="paper (2048/64, default), small (256/32), N:NT (sweep recipe), "
                         "readfloor, timeline, sweep, ragged or serve")
    ap.add_argument("--pool-bytes", type=float, default=1.0 * 2 ** 30,
                    help="total bytes of distinct pair copies the steps rotate over")
    ap.add_argument("--cpu-runs", type=int, default=10,
                    help="timed runs of the CPU oracle per configuration (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", choices=("auto", "yes", "no"), default="auto",
                    help="time the K steps as one graph replay (yes), as K eager launches "
                         "queued behind the prelude (no), or eager up to 64 steps and a graph "
                         "above (auto: a graph replay's own start-up costs about 10 us, "
                         "which weighs on a few launches; eager launches need about 11 us "
                         "of host time each, which a long run cannot hide)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements of the default run (read floor and "
                         "ceiling, separate kernels, batches, serving)")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: a few eager launches plus a 256 MiB copy of known size")
    ap.add_argument("--serve-rates", default="2000,10000,50000",
                    help="Poisson request rates of the serving leg of the default run ('' skips)")
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--rates", default="2000,5000,10000,20000,50000",
                    help="request rates of --workload serve (device-resident snapshots)")
    ap.add_argument("--h2d-rates", default="500,1000,2000",
                    help="request rates of --workload serve with pinned host snapshots")
    ap.add_argument("--sweep-launches", type=int, default=200,
                    help="launches per graph for --workload sweep and readfloor")
    ap.add_argument("--cells", default="",
                    help="--workload sweep: N:NT cells to run (default: all 20)")
    ap.add_argument("--shape", default="paper",
                    help="--workload readfloor / timeline: the pair shape (paper, small or N:NT); "
                         "for timeline also 'read', the plain read of the paper shape's bytes")
    ap.add_argument("--plan-out", default="",
                    help="write the launch plan (for a rocprofv3 trace summary) to this file")
    return ap.parse_args(argv)


def workload_spec(name: str):
    from paper_2501_10653_amd import synth
    if name == "paper":
        return synth.spec_paper_shape()
    if name == "small":
        return synth.spec_small()
    N, NT = (int(v) for v in name.split(":"))
    return synth.spec_sweep(N, NT)


def source_digest() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_record(N: int, NT: int, cfg: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, valid only
    while the kernel source and launch shape are the ones the counters were
    taken on."""
    path = os.path.join(PROFILES, f"traffic_iqa_tiles_{N}_nt{NT}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest() or rec.get("launch_cfg") != cfg:
        return None
    return rec


def _oracle_runs(x, y, NT: int, runs: int, threads: Optional[int] = None) -> dict:
    """`runs` timed calls of the FP64 oracle on one pair (after one untimed
    call), on `threads` OpenMP threads (None: all); median, min and p90."""
    from oracle import oracle
    c = oracle.f32const(1e-6)
    keep = oracle.num_threads()
    if threads is not None:
        oracle.set_num_threads(threads)
    try:
        used = oracle.num_threads()
        oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)
            ts.append(time.perf_counter() - t0)
    finally:
        oracle.set_num_threads(keep)
    t = np.array(ts)
    N = x.shape[0]
    med = float(np.median(t))
    return {"N": N, "NT": NT, "threads": used, "runs": runs,
            "median_ms": round(med * 1e3, 4), "min_ms": round(float(t.min()) * 1e3, 4),
            "p90_ms": round(float(np.percentile(t, 90)) * 1e3, 4),
            "GBs": round(8 * N * N / med / 1e9, 4),
            "tiles_per_s": round((N // NT) ** 2 / med, 1)}


def cpu_baseline(x, y, NT, runs: int, gpu_lisi: np.ndarray, gpu_aug: np.ndarray) -> dict:
    """The FP64 oracle, as it stands, timed on the host cores: the median of
    `runs` runs on the headline pair (all threads, and one thread), then the
    small configuration (256^2 / 32) and the corners of the size sweep
    (1024^2 and 8192^2 at N_T 16 and 256; one generated pair per N, since the
    oracle's time does not depend on the pixel values).  Its output on the
    headline pair also checks the last timed GPU result (LISI relative error,
    augLISI error relative to max(|augLISI|, P/(Sx+Sy+C)))."""
    from oracle import oracle
    from paper_2501_10653_amd import synth
    t_all = time.perf_counter()
    c = oracle.f32const(1e-6)
    ol, oa, _ = oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)
    head = _oracle_runs(x, y, NT, runs)
    one = _oracle_runs(x, y, NT, runs, threads=1)
    configs = [head, one]
    xs, ys, _ = synth.make_pair(synth.spec_small())
    configs += [_oracle_runs(xs, ys, 32, runs), _oracle_runs(xs, ys, 32, runs, threads=1)]
    for N in (1024, 8192):
        xc, yc, _ = synth.make_pair(synth.spec_sweep(N, 16))
        for nt in (16, 256):
            configs += [_oracle_runs(xc, yc, nt, runs), _oracle_runs(xc, yc, nt, runs, threads=1)]
        del xc, yc
    ol, oa = ol.ravel(), oa.ravel()
    gl = gpu_lisi.astype(np.float64).ravel()
    ga = gpu_aug.astype(np.float64).ravel()
    lisi_rel = np.abs(gl - ol) / np.where(ol != 0, np.abs(ol), 1.0)
    aug_err = np.abs(ga - oa) / np.maximum(np.abs(oa), np.abs(1.0 - oa))
    N = x.shape[0]
    return {
        "value": head["GBs"],
        "unit": "GB/s",
        "cores": head["threads"],
        "kind": "oracle",
        "tiles_per_s": head["tiles_per_s"],
        "ms_per_pair": head["median_ms"],
        "sample": f"FP64 C oracle (OpenMP over tile rows), median of {runs} runs on the "
                  f"{N}x{N} / {NT} pair; single thread and the other configurations in "
                  f"'configs' ({time.perf_counter() - t_all:.1f} s in all)",
        "single_thread": one,
        "configs": configs,
        "parity_of_last_gpu_step": {"lisi_max_rel": float(lisi_rel.max()),
                                    "aug_max_err": float(aug_err.max()),
                                    "pass_1e-5": bool(lisi_rel.max() <= 1e-5
                                                      and aug_err.max() <= 1e-5)},
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class ServingWorld:
    """Serving workload: 16 resident references with N round-robin over
    1024/2048/4096, a pool of device-resident snapshots per reference (the
    faintest sources gone, fresh noise), requests picking a reference
    uniformly and N_T uniformly from {32, 64}."""

    def __init__(self, torch, dev, snapshots_per_ref: int = 2, seed: int = 11):
        from paper_2501_10653_amd import synth
        self.torch = torch
        self.specs = synth.serving_references(count=16, seed=seed)
        self.refs, self.snaps = [], []
        for sp in self.specs:
            x, _, _ = synth.make_pair(sp)
            self.refs.append(torch.from_numpy(x).to(dev))
            self.snaps.append([torch.from_numpy(synth.make_snapshot(sp, k)).to(dev)
                               for k in range(snapshots_per_ref)])
        self.host_snaps = None

    def pin_snapshots(self):
        """Pinned host copies of the snapshots, for the H2D serving mode."""
        if self.host_snaps is None:
            self.host_snaps = [[s.cpu().pin_memory() for s in per] for per in self.snaps]

    def requests(self, srv, ids, count: int, seed: int, host: bool = False):
        rng = np.random.default_rng((seed, 3))
        out, nbytes = [], 0
        snaps = self.host_snaps if host else self.snaps
        for i in range(count):
            r = int(rng.integers(len(self.refs)))
            k = int(rng.integers(len(snaps[r])))
            NT = int(rng.choice([32, 64]))
            # every snapshot is complete before the replay starts (run_serving
            # synchronises the device), so the batches need no ready event
            out.append(srv.request(snaps[r][k], ids[r], NT, ready=False))
            nbytes += 8 * self.specs[r].N ** 2
        return out, nbytes


def run_serving(torch, world, rate: float, seconds: float, budget: int = 16 << 30,
                streams: Optional[int] = None, max_batch: int = 512, seed: int = 0,
                host: bool = False) -> dict:
    """One open-loop serving run.  Launch slots default to 4 for device-resident
    snapshots (more batches in flight cut the tail at high rates) and 2 for
    host snapshots (their copies share one PCIe link, so more slots in flight
    only stretch each batch)."""
    from paper_2501_10653_amd import synth
    if streams is None:
        streams = 2 if host else 4
    from paper_2501_10653_amd.serve import Server, latency_summary
    count = max(200, int(rate * seconds))
    log(f"serving {rate:.0f} req/s ({'host' if host else 'device'} snapshots)")
    arena = (2 << 30) if host else 0
    if host:
        world.pin_snapshots()
    with Server(budget, streams=streams, max_batch=max_batch, host_arena_bytes=arena) as srv:
        ids = [srv.add_reference(r) for r in world.refs]
        reqs, nbytes = world.requests(srv, ids, count, seed, host=host)
        torch.cuda.synchronize()
        arrivals = synth.poisson_arrivals(rate, count, seed=seed)
        comps = srv.replay(reqs, arrivals, timeout_s=120.0)
        st = srv.stats()
    summ = latency_summary(comps)
    summ.update({"offered_rps": rate, "requests": count, "batches": st["batches"],
                 "snapshots": "pinned host (H2D per request)" if host else "device-resident",
                 "max_batch": st["max_batch"],
                 "peak_in_flight_MiB": round(st["peak_in_flight_bytes"] / 2 ** 20, 1),
                 "budget_GiB": budget / 2 ** 30, "streams": streams,
                 "GBs_delivered": round(nbytes * summ.get("throughput_rps", 0) / count / 1e9, 1)})
    for k in ("p50_us", "p99_us", "max_us", "mean_us", "p50_done_us", "p99_done_us",
              "throughput_rps", "span_s"):
        if k in summ:
            summ[k] = round(summ[k], 2)
    return summ


def ragged_pairs(torch, dev, count: int = 256, seed: int = 7):
    """The ragged-batch workload's pairs: one prototype pair per (N, transient
    or not), copied into distinct device buffers for every pair (timing is
    content-independent)."""
    from paper_2501_10653_amd import synth
    specs = synth.ragged_specs(count=count, seed=seed)
    proto = {}
    for N in sorted({sp.N for sp in specs}):
        for kind in (0, 1):
            sp = synth.PairSpec(N=N, NT=64, n_src=synth.scaled_count(33, N, 1), amp_lo=1e-3,
                                amp_hi=2.0, fwhm=4.0, noise_sigma=1e-4,
                                n_drop=3 if kind else 0, seed=N * 10 + kind)
            x, y, _ = synth.make_pair(sp)
            proto[(N, kind)] = (torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    pairs = []
    for sp in specs:
        x, y = proto[(sp.N, 1 if sp.n_drop else 0)]
        pairs.append((x.clone(), y.clone(), sp.NT))
    del proto
    return pairs


def run_ragged(torch, dev, count: int = 256, seed: int = 7) -> dict:
    """Ragged batch: `count` pairs with N uniform over {512, 1024, 2048, 4096}
    and N_T over {32, 64, 128}, 20% with 1-5 faintest sources removed and the
    rest noise-only.  One prototype pair is generated per (N, kind) and copied
    into distinct device buffers for every pair (timing is content-independent).
    Times one persistent launch (eager, and in a graph) against `count`
    single-pair launches with their tuned shapes (eager, and in a graph), each
    the median of 5 timed runs after a prelude."""
    from paper_2501_10653_amd import iqa_tiles
    from paper_2501_10653_amd.batch import Batch
    from paper_2501_10653_amd.measure import GraphTimer
    pairs = ragged_pairs(torch, dev, count, seed)
    total = sum(8 * p[0].shape[0] ** 2 for p in pairs)
    s = torch.cuda.Stream(dev)
    timer = GraphTimer(torch, dev, s)

    def eager_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            timer.run_prelude(1e-3)
            e0.record(s)
            fn()
            e1.record(s)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    b = Batch(pairs)
    out = {"pairs": count, "bytes": total, "units": b.units, "waves": b.waves}
    out["batched_eager_ms"] = round(eager_ms(lambda: b.run(stream=s)), 4)
    g = b.capture(s)
    ms = float(np.median(timer.replay_ms(g, reps=5)))
    out["batched_graph_ms"] = round(ms, 4)
    out["batched_graph_GBs"] = round(total / ms / 1e6, 1)
    outs = [(torch.empty(p[0].shape[0] // p[2], p[0].shape[0] // p[2], device=dev),
             torch.empty(p[0].shape[0] // p[2], p[0].shape[0] // p[2], device=dev))
            for p in pairs]

    def plain():
        for (x, y, NT), (lo, ao) in zip(pairs, outs):
            iqa_tiles(x, y, NT, out={"lisi": lo, "auglisi": ao}, stream=s)

    ms = eager_ms(plain)
    out["plain_eager_ms"] = round(ms, 4)
    out["plain_eager_GBs"] = round(total / ms / 1e6, 1)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        plain()
    ms = float(np.median(timer.replay_ms(g2, reps=5)))
    out["plain_graph_ms"] = round(ms, 4)
    out["plain_graph_GBs"] = round(total / ms / 1e6, 1)
    out["hbm_frac_batched"] = round(out["batched_graph_GBs"] / HBM_PEAK_GBS, 4)
    out["batched_vs_plain_graph"] = round(out["plain_graph_ms"] / out["batched_graph_ms"], 3)
    del g, g2, b, pairs
    torch.cuda.empty_cache()
    return out


def run_readfloor(torch, dev, args) -> dict:
    """Plain reads and empty launches of the headline pair's byte count, in
    many shapes, beside the fused kernel timed the same way."""
    from paper_2501_10653_amd import default_cfg, iqa_tiles, synth
    from paper_2501_10653_amd.measure import GraphTimer, Plan, read_floor
    from paper_2501_10653_amd.tune import device_copies
    plan = Plan()
    spec = workload_spec(args.shape)
    N, NT = spec.N, spec.NT
    nbytes = 8 * N * N
    K = args.sweep_launches
    floor = read_floor(torch, dev, nbytes, K=K, pool_bytes=args.pool_bytes, plan=plan)
    x, y, _ = synth.make_pair(spec)
    pool = max(2, int(math.ceil(args.pool_bytes / nbytes)))
    xs = device_copies(torch, dev, x, pool)
    ys = device_copies(torch, dev, y, pool)
    stream = torch.cuda.Stream(dev)
    timer = GraphTimer(torch, dev, stream)
    cfg = default_cfg(N, NT, xs[0], ys[0])
    ns = N // NT
    out = {"lisi": torch.empty(ns, ns, device=dev), "auglisi": torch.empty(ns, ns, device=dev)}
    us = timer.per_launch_us(lambda i: iqa_tiles(xs[i % pool], ys[i % pool], NT, out=out,
                                                 cfg=cfg, stream=stream), K)
    plan.add(f"fused {N}^2/{NT} (warm)", "tiles_kernel", K, bytes=nbytes)
    plan.add(f"fused {N}^2/{NT}", "tiles_kernel", K, bytes=nbytes)
    if args.plan_out:
        plan.dump(args.plan_out)
    best = floor["fastest_read"]
    return {"metric": f"plain-read floor of one {nbytes}-byte launch", "unit": "us",
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": f"{nbytes} B per launch (a {N}^2 FP32 pair), "
                                   f"{K} launches per graph over {floor['pool_buffers']} "
                                   f"distinct buffers"},
            "fused": {"cfg": cfg, "us": round(us, 3), "GBs": round(nbytes / us / 1e3, 1),
                      "vs_fastest_read": round(best["us"] / us, 4)},
            "fastest_read": best, "fastest_empty": floor["fastest_empty"],
            "rows": floor["rows"]}


def run_timeline(torch, dev, args) -> dict:
    from paper_2501_10653_amd import default_cfg, synth
    from paper_2501_10653_amd.measure import QUICK_READS, read_timeline, timeline
    from paper_2501_10653_amd.tune import device_copies
    if args.shape == "read":
        # the plain read of the paper-shape pair's bytes, in the shape that came
        # out fastest in the read-floor sweep
        _, blocks, threads, loads = QUICK_READS[0]
        nbytes = 8 * workload_spec("paper").N ** 2
        res = read_timeline(torch, dev, nbytes, blocks, threads, loads, launches=64,
                            pool_bytes=args.pool_bytes)
        return {"metric": "per-workgroup timeline of the plain read", "unit": "us",
                "n_gpus": 1, "data": "synthetic",
                "config": {"workload": f"{nbytes} B per launch, {blocks} workgroups x {threads} "
                                       f"threads, {loads} loads in flight per lane, 64 "
                                       f"back-to-back launches in a graph"},
                "timeline": res}
    spec = workload_spec(args.shape)
    x, y, _ = synth.make_pair(spec)
    nbytes = 8 * spec.N ** 2
    pool = max(2, int(math.ceil(args.pool_bytes / nbytes)))
    xs = device_copies(torch, dev, x, pool)
    ys = device_copies(torch, dev, y, pool)
    cfg = default_cfg(spec.N, spec.NT, xs[0], ys[0])
    res = timeline(torch, dev, xs, ys, spec.NT, cfg, launches=64)
    return {"metric": "per-workgroup timeline of the fused launch", "unit": "us",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": f"{spec.N}^2 / {spec.NT}, 64 back-to-back launches in a "
                                   f"graph over {pool} distinct pairs"},
            "timeline": res}


def run_sweep(torch, dev, args) -> dict:
    """Every cell of the size sweep (N in 1024..8192, N_T in 16..256) with its
    default launch shape, K launches per graph over >= 1 GiB of distinct
    copies, timed with events (median of 3 replays)."""
    from paper_2501_10653_amd import default_cfg, iqa_tiles, prepare, synth
    from paper_2501_10653_amd.measure import GraphTimer, Plan
    from paper_2501_10653_amd.tune import device_copies
    plan = Plan()
    cells = SWEEP_CELLS
    if args.cells:
        cells = [tuple(int(v) for v in c.split(":")) for c in args.cells.split(",")]
    K = args.sweep_launches
    stream = torch.cuda.Stream(dev)
    timer = GraphTimer(torch, dev, stream)
    rows = []
    pairs = {}
    for N, NT in cells:
        if N not in pairs:
            pairs.clear()
            torch.cuda.empty_cache()
            x, y, _ = synth.make_pair(synth.spec_sweep(N, 64))
            pool = max(2, int(math.ceil(args.pool_bytes / (8 * N * N))))
            pairs[N] = (device_copies(torch, dev, x, pool), device_copies(torch, dev, y, pool))
        xs, ys = pairs[N]
        pool = len(xs)
        cfg = default_cfg(N, NT, xs[0], ys[0])
        prepare(N, NT, cfg, stream=stream)      # the split workspace, before capture
        ns = N // NT
        out = {"lisi": torch.empty(ns, ns, device=dev),
               "auglisi": torch.empty(ns, ns, device=dev)}
        g = timer.capture(lambda i: iqa_tiles(xs[i % pool], ys[i % pool], NT, out=out, cfg=cfg,
                                              stream=stream), K)
        ms = timer.replay_ms(g, reps=3)
        del g
        us = float(np.median(ms)) * 1e3 / K
        nbytes = 8 * N * N
        plan.add(f"{N}^2/{NT} (warm)", "tiles_kernel", K, bytes=nbytes)
        for r in range(3):
            plan.add(f"{N}^2/{NT}" + ("" if r == 0 else f" (rep {r + 1})"), "tiles_kernel", K,
                     bytes=nbytes)
        rows.append({"N": N, "NT": NT, "cfg": cfg, "us": round(us, 3),
                     "GBs": round(nbytes / us / 1e3, 1),
                     "frac_of_peak": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 4)})
        print(json.dumps({"cell": f"{N}x{NT}", "us": round(us, 3)}), file=sys.stderr, flush=True)
    if args.plan_out:
        plan.dump(args.plan_out)
    return {"metric": "fused kernel time per size-sweep cell", "unit": "us",
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": f"size sweep, {K} launches per graph per cell, distinct "
                                   f"copies >= {args.pool_bytes / 2 ** 30:.0f} GiB"},
            "cells": rows}


def main(argv=None) -> int:
    args = parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (--gpus 1); the path "
                                   "is single-GPU and no multi-GPU launch is provided"}))
        return 2

    import torch
    from paper_2501_10653_amd import default_cfg, iqa_tiles, synth
    from paper_2501_10653_amd.iqa import auglisi_tiles, lisi_tiles, read_ceiling
    from paper_2501_10653_amd.measure import GraphTimer
    from paper_2501_10653_amd.tune import device_copies

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}))
        return 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    special = {"readfloor": run_readfloor, "timeline": run_timeline, "sweep": run_sweep}
    if args.workload in special:
        print(json.dumps(special[args.workload](torch, dev, args)), flush=True)
        return 0

    if args.workload == "ragged" and args.profile:
        # Counter runs: three eager launches of the batch, then a copy of known
        # size (256 MiB read + 256 MiB written) that calibrates the counters.
        from paper_2501_10653_amd.batch import Batch
        pairs = ragged_pairs(torch, dev)
        b = Batch(pairs)
        for _ in range(3):
            b.run()
        src = torch.empty(64 * 2 ** 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": True, "workload": "ragged", "pairs": len(pairs),
                          "bytes": sum(8 * p[0].shape[0] ** 2 for p in pairs),
                          "units": b.units, "waves": b.waves}), flush=True)
        return 0

    if args.workload == "ragged":
        r = run_ragged(torch, dev)
        print(json.dumps({"metric": "ragged batch HBM GB/s (one persistent launch, graph)",
                          "value": r["batched_graph_GBs"], "unit": "GB/s",
                          "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
                          "data": "synthetic",
                          "config": {"workload": "256 FP32 pairs, N in {512..4096}, "
                                                 "N_T in {32, 64, 128}"},
                          "detail": r}), flush=True)
        return 0

    if args.workload == "serve":
        world = ServingWorld(torch, dev)
        rows = [run_serving(torch, world, float(r), args.serve_seconds, seed=i)
                for i, r in enumerate(args.rates.split(","))]
        rows += [run_serving(torch, world, float(r), args.serve_seconds, seed=100 + i, host=True)
                 for i, r in enumerate(args.h2d_rates.split(",")) if r]
        print(json.dumps({"metric": "p99 request latency (serving, device-resident snapshots)",
                          "unit": "us", "higher_is_better": False, "n_gpus": 1,
                          "data": "synthetic",
                          "config": {"workload": "16 resident references (N 1024/2048/4096), "
                                                 "snapshots vs reference, N_T in {32, 64}, "
                                                 "Poisson arrivals"},
                          "rates": rows}), flush=True)
        return 0

    spec = workload_spec(args.workload)
    N, NT = spec.N, spec.NT
    ns = N // NT
    x, y, _ = synth.make_pair(spec)
    bytes_pair = 8 * N * N
    pool = max(2, int(math.ceil(args.pool_bytes / bytes_pair)))
    xs = device_copies(torch, dev, x, pool)
    ys = device_copies(torch, dev, y, pool)
    lisi = torch.empty(ns, ns, device=dev)
    aug = torch.empty(ns, ns, device=dev)
    out = {"lisi": lisi, "auglisi": aug}
    cfg = default_cfg(N, NT, xs[0], ys[0])
    stream = torch.cuda.Stream(dev)

    def step(i):
        iqa_tiles(xs[i % pool], ys[i % pool], NT, out=out, cfg=cfg, stream=stream)

    if args.profile:
        # A handful of eager launches for counters, then a copy of known size
        # (256 MiB read + 256 MiB written) that calibrates the byte counters.
        with torch.cuda.stream(stream):
            for i in range(max(args.steps, 1)):
                step(i)
            src = torch.empty(64 * 2 ** 20, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": True, "N": N, "NT": NT, "launches": max(args.steps, 1),
                          "copy_bytes": src.numel() * 4}), flush=True)
        return 0

    # warm-up (eager), then capture exactly K launches into one graph
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            step(i)
    torch.cuda.synchronize()

    K = args.steps
    use_graph = args.graph == "yes" or (args.graph == "auto" and K > EAGER_MAX_STEPS)
    if args.plan_out:
        from paper_2501_10653_amd.measure import Plan
        plan = Plan()
        kname = "tiles_kernel<"
        plan.add("warm-up (eager)", kname, args.warmup, bytes=bytes_pair)
        plan.add("untimed pass", kname, K, bytes=bytes_pair)
        plan.add("timed steps", kname, K, bytes=bytes_pair)
        plan.dump(args.plan_out)
    timer = GraphTimer(torch, dev, stream)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    if use_graph:
        graph = timer.capture(step, K)
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            graph.replay()                  # one untimed replay
        host_s = time.perf_counter() - t0
        torch.cuda.synchronize()
    else:
        t0 = time.perf_counter()            # one untimed pass: the host's enqueue time
        for i in range(K):
            step(i)
        host_s = time.perf_counter() - t0
        torch.cuda.synchronize()
    # The timed region: K launches already queued behind the prelude.
    torch.cuda.synchronize()
    timer.run_prelude(host_s)
    wall0 = time.perf_counter()
    t_start.record(stream)
    if use_graph:
        with torch.cuda.stream(stream):
            graph.replay()
    else:
        for i in range(K):
            step(i)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / K
    # algorithmic HBM bytes of one step: both images read once, the two IQA
    # matrices written once
    bytes_step = bytes_pair + 2 * 4 * ns * ns
    gbs = bytes_step / (ms_step * 1e-3) / 1e9

    log(f"headline: {ms_step * 1e3:.3f} us per launch over {K} launches")
    gpu_lisi = lisi.cpu().numpy()
    gpu_aug = aug.cpu().numpy()
    if use_graph:
        del graph

    extras, batched, floor = {}, None, None
    if not args.no_extras:
        log("read floor (quick)")
        fo = {"lisi": torch.empty(ns, ns, device=dev), "auglisi": torch.empty(ns, ns, device=dev)}
        floor = quick_read_floor(
            torch, dev, bytes_pair, args.pool_bytes,
            lambda i, s: iqa_tiles(xs[i % pool], ys[i % pool], NT, out=fo, cfg=cfg, stream=s))
        log("read ceiling, separate kernels")
        extras = run_extras(torch, dev, xs, ys, N, NT, pool, stream, read_ceiling,
                            lisi_tiles, auglisi_tiles, iqa_tiles, cfg, bytes_pair)
        extras["kernel_frac_of_read_ceiling"] = round(gbs / extras["read_ceiling_gbs"], 4)
        log("same-shape batch")
        batched = run_same_shape_batch(torch, xs, ys, NT, stream, bytes_pair, ms_step)
        batched["frac_of_read_ceiling"] = round(batched["gbs"] / extras["read_ceiling_gbs"], 4)

    traffic = traffic_record(N, NT, cfg)
    roofline = {
        "bound": "hbm",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": (traffic["hbm_bytes_per_launch"] if traffic else None),
    }
    line = {
        "metric": METRIC,
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"fused LISI+augLISI, one {N}x{N} FP32 image pair, {NT}x{NT} tiles "
                        f"({ns}x{ns} IQA matrix); beam-convolved sources on noise",
            "N": N, "NT": NT, "pool_pairs": pool, "launch_cfg": cfg,
            "graph": use_graph,
        },
        "tiles_per_s": round(ns * ns / (ms_step * 1e-3), 1),
        "bytes_per_step": bytes_step,
        "hbm_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
        "wall_s_timed": round(wall, 4),
        "roofline": roofline,
    }
    if floor:
        line["reference_read"] = {**floor,
                                  "headline_step_frac_of_fastest_read":
                                      round(floor["fastest_read"]["us"] / (ms_step * 1e3), 4)}
    if extras:
        line["extras"] = extras
    if batched:
        line["batched"] = batched
    del xs, ys
    torch.cuda.empty_cache()
    if not args.no_extras and args.workload == "paper":
        log("ragged batch")
        line["ragged"] = run_ragged(torch, dev)
    if args.serve_rates and not args.no_extras and args.workload == "paper":
        log("serving")
        world = ServingWorld(torch, dev)
        line["serving"] = [run_serving(torch, world, float(r), args.serve_seconds, seed=i)
                           for i, r in enumerate(args.serve_rates.split(","))]
        del world
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(x, y, NT, args.cpu_runs, gpu_lisi, gpu_aug)
        line["cpu_baseline"]["cpu_model"] = cpu_model()
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


def quick_read_floor(torch, dev, nbytes: int, pool_bytes: float, fused) -> dict:
    """A few shapes of the plain read of the same bytes per launch (the ones
    that came out fastest in the full read-floor sweep): what a launch of this
    size can reach on this GPU.  `fused(i, stream)` launches the fused kernel
    on the i-th pair, which is timed the same way right after (200 launches
    in one graph replay), so that the two compare like for like."""
    from paper_2501_10653_amd.measure import GraphTimer, read_floor
    K = 200
    res = read_floor(torch, dev, nbytes, K=K, pool_bytes=pool_bytes, quick=True)
    stream = torch.cuda.Stream(dev)
    timer = GraphTimer(torch, dev, stream)
    us = timer.per_launch_us(lambda i: fused(i, stream), K, reps=3)
    best = res["fastest_read"]
    return {"fastest_read": best, "fastest_empty": res["fastest_empty"],
            "shapes_timed": len(res["rows"]),
            "fused_same_harness_us": round(us, 3),
            "kernel_frac_of_fastest_read": round(best["us"] / us, 4)}


def run_extras(torch, dev, xs, ys, N, NT, pool, stream, read_ceiling, lisi_tiles,
               auglisi_tiles, iqa_tiles, cfg, bytes_pair) -> dict:
    """Read ceiling over 2 GiB, and the two separate kernels vs the fused one."""
    from paper_2501_10653_amd.measure import GraphTimer
    ex = {}
    timer = GraphTimer(torch, dev, stream)
    buf = torch.empty(512 * 2 ** 20, device=dev)      # 2 GiB
    buf.fill_(1.0)
    outc = torch.empty(8192, device=dev)
    us = timer.per_launch_us(lambda i: read_ceiling(buf, outc, stream=stream), 5, reps=3)
    ex["read_ceiling_gbs"] = round(buf.numel() * 4 / us / 1e3, 1)
    del buf
    ns = N // NT
    lo = torch.empty(ns, ns, device=dev)
    ao = torch.empty(ns, ns, device=dev)
    K = 400
    for name, fn in (("lisi_only", lambda i: lisi_tiles(xs[i % pool], ys[i % pool], NT, out=lo,
                                                         stream=stream)),
                     ("auglisi_only", lambda i: auglisi_tiles(xs[i % pool], ys[i % pool], NT,
                                                              out=ao, stream=stream)),
                     ("fused", lambda i: iqa_tiles(xs[i % pool], ys[i % pool], NT,
                                                   out={"lisi": lo, "auglisi": ao}, cfg=cfg,
                                                   stream=stream))):
        us = timer.per_launch_us(fn, K)
        ex[f"{name}_us"] = round(us, 3)
        ex[f"{name}_gbs"] = round(bytes_pair / us / 1e3, 1)
    ex["separate_total_us"] = round(ex["lisi_only_us"] + ex["auglisi_only_us"], 3)
    return ex


def run_same_shape_batch(torch, xs, ys, NT, stream, bytes_pair, single_ms, reps: int = 20) -> dict:
    """Every pair of the pool in one persistent batch launch (the ragged-batch
    kernel with all pairs of one shape), `reps` launches in one graph: the
    throughput of the same pairs when they come as a batch rather than one
    launch each, next to the single-launch value."""
    from paper_2501_10653_amd.batch import Batch
    from paper_2501_10653_amd.measure import GraphTimer
    b = Batch([(x, y, NT) for x, y in zip(xs, ys)])
    timer = GraphTimer(torch, xs[0].device, stream)
    us_launch = timer.per_launch_us(lambda i: b.run(stream=stream), reps)
    ms = us_launch / 1e3
    ns = xs[0].shape[0] // NT
    gbs = len(xs) * (bytes_pair + 2 * 4 * ns * ns) / (ms * 1e-3) / 1e9
    out = {"pairs_per_launch": len(xs), "launches": reps, "waves": b.waves,
           "us_per_launch": round(ms * 1e3, 2),
           "us_per_pair": round(ms * 1e3 / len(xs), 3),
           "gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
           "vs_single_launch": round(single_ms / (ms / len(xs)), 3)}
    del b
    return out


if __name__ == "__main__":
    sys.exit(main())
