#!/usr/bin/env python3
"""Benchmark of the fused tile-wise LISI + augLISI path on one MI355X.

A step is one fused launch (clamp, per-pixel terms, per-tile compensated
reduction, Eq. 1 and Eq. 2 finalisation) over one synthetic FP32 image pair of
the paper's shape: N = 2048, N_T = 64 (32 x 32 IQA matrix).  Inputs are
resident in HBM before the timed region.  Steps rotate over a pool of distinct
device copies of the pair (>= 1 GiB in total) so that no step is served from
the 256 MB Infinity Cache that the previous steps filled.  The K timed steps
are one replay of a HIP graph holding exactly K launches.

Prints one JSON line (rank 0).  ``--gpus N`` with N > 1 is not supported: this
is a single-GPU path.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fused LISI+augLISI HBM GB/s (% peak) at 2048²/NT64; p99 request latency"
HBM_PEAK_GBS = 8000.0       # MI355X published HBM3E bandwidth
KERNEL_SRC = os.path.join(ROOT, "paper_2501_10653_amd", "csrc", "iqa_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="paper",
                    help="paper (2048/64, default), small (256/32) or N:NT (sweep recipe)")
    ap.add_argument("--pool-bytes", type=float, default=1.0 * 2 ** 30,
                    help="total bytes of distinct pair copies the steps rotate over")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of a graph")
    ap.add_argument("--extras", action="store_true",
                    help="also time the read ceiling and the two separate kernels")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: a few eager launches plus a 256 MiB copy of known size")
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


def traffic_record(N: int, NT: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, valid only
    while the kernel source is the one the counters were taken on."""
    path = os.path.join(PROFILES, f"traffic_iqa_tiles_{N}_nt{NT}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest():
        return None
    return rec


def cpu_baseline(x, y, NT, seconds: float, bytes_pair: int, n_tiles: int,
                 gpu_lisi: np.ndarray, gpu_aug: np.ndarray) -> dict:
    """The FP64 oracle, as it stands, on the host cores: repeated over the same
    pair until ``seconds`` of wall time have passed.  Its output also checks
    the last timed GPU result (LISI relative error, augLISI error relative to
    max(|augLISI|, P/(Sx+Sy+C)))."""
    from oracle import oracle
    c = oracle.f32const(1e-6)
    ol, oa, _ = oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)       # also warms the caches
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.iqa_tiles(x, y, NT, c / 2, c, c, c)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    ol, oa = ol.ravel(), oa.ravel()
    gl = gpu_lisi.astype(np.float64).ravel()
    ga = gpu_aug.astype(np.float64).ravel()
    lisi_rel = np.abs(gl - ol) / np.where(ol != 0, np.abs(ol), 1.0)
    aug_err = np.abs(ga - oa) / np.maximum(np.abs(oa), np.abs(1.0 - oa))
    return {
        "value": round(bytes_pair * reps / el / 1e9, 4),
        "unit": "GB/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "tiles_per_s": round(n_tiles * reps / el, 1),
        "ms_per_pair": round(el / reps * 1e3, 3),
        "sample": f"FP64 C oracle (OpenMP over tile rows) on the same {x.shape[0]}x{x.shape[0]} "
                  f"pair, {reps} repetitions in {el:.1f} s",
        "parity_of_last_gpu_step": {"lisi_max_rel": float(lisi_rel.max()),
                                    "aug_max_err": float(aug_err.max()),
                                    "pass_1e-5": bool(lisi_rel.max() <= 1e-5
                                                      and aug_err.max() <= 1e-5)},
    }


def main(argv=None) -> int:
    args = parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU path: run with --gpus 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        return 2

    import torch
    from paper_2501_10653_amd import default_cfg, iqa_tiles, synth
    from paper_2501_10653_amd.iqa import auglisi_tiles, lisi_tiles, read_ceiling

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device visible"}))
        return 1
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    spec = workload_spec(args.workload)
    N, NT = spec.N, spec.NT
    ns = N // NT
    x, y, _ = synth.make_pair(spec)
    bytes_pair = 8 * N * N
    pool = max(2, int(math.ceil(args.pool_bytes / bytes_pair)))
    xs = [torch.from_numpy(x).to(dev) for _ in range(1)]
    ys = [torch.from_numpy(y).to(dev) for _ in range(1)]
    for _ in range(pool - 1):
        xs.append(xs[0].clone())
        ys.append(ys[0].clone())
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
    use_graph = not args.no_graph
    graph = None
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            for i in range(K):
                step(i)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()                  # one untimed replay
        torch.cuda.synchronize()

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    if use_graph:
        with torch.cuda.stream(stream):
            graph.replay()
    else:
        with torch.cuda.stream(stream):
            for i in range(K):
                step(i)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / K
    gbs = bytes_pair / (ms_step * 1e-3) / 1e9

    gpu_lisi = lisi.cpu().numpy()
    gpu_aug = aug.cpu().numpy()

    extras = {}
    if args.extras:
        extras = run_extras(torch, dev, xs, ys, N, NT, pool, stream, read_ceiling,
                            lisi_tiles, auglisi_tiles, iqa_tiles, cfg, bytes_pair)

    traffic = traffic_record(N, NT)
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
        "hbm_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
        "wall_s_timed": round(wall, 4),
        "roofline": roofline,
    }
    if extras:
        line["extras"] = extras
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, y, NT, args.cpu_seconds, bytes_pair, ns * ns,
                                            gpu_lisi, gpu_aug)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    return 0


def run_extras(torch, dev, xs, ys, N, NT, pool, stream, read_ceiling, lisi_tiles,
               auglisi_tiles, iqa_tiles, cfg, bytes_pair) -> dict:
    """Read ceiling over >= 2 GiB, and the two separate kernels vs the fused one."""
    ex = {}
    buf = torch.empty(512 * 2 ** 20, device=dev)      # 2 GiB
    buf.fill_(1.0)
    outc = torch.empty(8192, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        for _ in range(3):
            read_ceiling(buf, outc, stream=stream)
        best = []
        for _ in range(5):
            ev0.record(stream)
            read_ceiling(buf, outc, stream=stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            best.append(ev0.elapsed_time(ev1))
    ms = min(best)
    ex["read_ceiling_gbs"] = round(buf.numel() * 4 / (ms * 1e-3) / 1e9, 1)
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
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for i in range(K):
                fn(i)
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
        ev0.record(stream)
        with torch.cuda.stream(stream):
            g.replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / K
        ex[f"{name}_us"] = round(ms * 1e3, 3)
        ex[f"{name}_gbs"] = round(bytes_pair / (ms * 1e-3) / 1e9, 1)
    ex["separate_total_us"] = round(ex["lisi_only_us"] + ex["auglisi_only_us"], 3)
    return ex


if __name__ == "__main__":
    sys.exit(main())
