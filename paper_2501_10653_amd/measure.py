"""Measurement harness: timed graph replays, the read floor of a launch size,
per-workgroup timelines, and launch plans for rocprofv3 summaries.

Timing rule used throughout: a HIP graph of K launches is captured, replayed
once untimed, and replayed again between two events on the launch stream.
Before the timed replay the stream gets a few plain reads of a 512 MiB
scratch buffer (a *prelude*): they keep the GPU busy while the host enqueues
the start event and the graph, so the timed region starts with all K launches
already queued (it measures the GPU's back-to-back launch rate, not the
host's submission latency), and they push whatever the Infinity Cache held
out of it.  The prelude only reads: writes would leave dirty lines in the
caches whose write-back then competes with the timed launches (measured: a
prelude of fills slows 2048^2 launches by 0.3-0.5 us each, even 2000 launches
later).
"""

from __future__ import annotations

import json
import math
import sys
import time
from typing import Callable, Dict, List, Optional

import numpy as np

HBM_PEAK_GBS = 8000.0
PRELUDE_BYTES = 512 << 20        # one prelude read: ~0.1 ms of HBM reads
PRELUDE_READ_S = 100e-6
PRELUDE_BLOCKS = 1024


class Plan:
    """The sequence of launches a measurement makes, for matching a rocprofv3
    kernel trace to its segments: each segment is `count` dispatches of a
    kernel whose name contains `kernel`, in launch order."""

    def __init__(self):
        self.segments: List[dict] = []

    def add(self, label: str, kernel: str, count: int, **info) -> None:
        self.segments.append({"label": label, "kernel": kernel, "count": int(count), **info})

    def dump(self, path: str) -> None:
        with open(path, "w") as fh:
            json.dump({"segments": self.segments}, fh, indent=1)


class GraphTimer:
    """Event timing of graph replays on one stream, with a prelude."""

    def __init__(self, torch, dev, stream):
        self.torch = torch
        self.stream = stream
        self.prelude = torch.ones(PRELUDE_BYTES // 4, device=dev)
        self.prelude_out = torch.empty(PRELUDE_BLOCKS, device=dev)
        torch.cuda.synchronize()

    def run_prelude(self, host_s: float) -> None:
        from .iqa import probe_read
        from ._lib import PROBE_READ_REGS
        reads = int(min(64, max(2, math.ceil(2.0 * host_s / PRELUDE_READ_S))))
        for _ in range(reads):
            probe_read(self.prelude, self.prelude_out, 256, 8, PROBE_READ_REGS,
                       stream=self.stream)

    def capture(self, launch: Callable[[int], None], K: int):
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            for i in range(K):
                launch(i)
        torch.cuda.synchronize()
        return g

    def replay_ms(self, graph, reps: int = 1) -> List[float]:
        """Untimed replay (also measures the host's submission time), then
        `reps` timed replays, each after a prelude; ms per replay."""
        torch = self.torch
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            graph.replay()
        host_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            self.run_prelude(host_s)
            e0.record(self.stream)
            with torch.cuda.stream(self.stream):
                graph.replay()
            e1.record(self.stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    def per_launch_us(self, launch: Callable[[int], None], K: int, reps: int = 1) -> float:
        g = self.capture(launch, K)
        ms = self.replay_ms(g, reps)
        del g
        return float(np.median(ms)) * 1e3 / K


def distinct_buffers(torch, dev, nbytes: int, pool_bytes: float) -> list:
    n = max(2, int(math.ceil(pool_bytes / nbytes)))
    bufs = [torch.empty(nbytes // 4, device=dev) for _ in range(n)]
    for b in bufs:
        b.fill_(1.0)
    return bufs


# ---------------------------------------------------------------------------
# Read floor
# ---------------------------------------------------------------------------

READ_MODES = {0: "regs (args preloaded)", 1: "regs (args loaded)", 2: "direct-to-LDS"}

# (mode, workgroups, threads, loads in flight per lane): the shapes that came
# out fastest for a 32 MiB launch in the full sweep, for a short run.
QUICK_READS = [(0, 256, 512, 4), (1, 256, 512, 4), (0, 512, 256, 4), (0, 512, 512, 4),
               (0, 1024, 256, 8), (0, 2048, 256, 4), (2, 512, 512, 8)]


def read_floor(torch, dev, nbytes: int, K: int = 200, pool_bytes: float = 1.0 * 2 ** 30,
               plan: Optional[Plan] = None, quick: bool = False) -> Dict:
    """Plain reads of exactly `nbytes` per launch in many shapes, and the empty
    launch, each timed as K launches in one graph over distinct buffers.
    Returns every shape's µs per launch and the fastest read."""
    from .iqa import probe_empty, probe_read
    stream = torch.cuda.Stream(dev)
    timer = GraphTimer(torch, dev, stream)
    bufs = distinct_buffers(torch, dev, nbytes, pool_bytes)
    pool = len(bufs)
    n4 = nbytes // 16
    rows = []

    empties = [(1, 64), (256, 256), (512, 256), (1024, 256), (256, 1024)]
    for blocks, threads in empties:
        us = timer.per_launch_us(lambda i: probe_empty(blocks, threads, stream=stream), K)
        rows.append({"kind": "empty", "blocks": blocks, "threads": threads, "us": round(us, 3)})
        if plan:
            plan.add(f"empty b{blocks} t{threads} (warm)", "probe_empty", K)
            plan.add(f"empty b{blocks} t{threads}", "probe_empty", K)

    if quick:
        shapes = QUICK_READS
    else:
        shapes = [(mode, blocks, threads, loads) for mode in (0, 1, 2)
                  for blocks in (256, 512, 1024, 2048, 4096) for threads in (256, 512, 1024)
                  for loads in (4, 8, 16, 32)]
    kname = {0: "probe_read_regs<", 1: "probe_read_regs_struct<", 2: "probe_read_lds<"}
    said = None
    for mode, blocks, threads, loads in shapes:
        if (mode, blocks) != said:
            print(f"[read floor] {READ_MODES[mode]}, {blocks} workgroups", file=sys.stderr,
                  flush=True)
            said = (mode, blocks)
        per = math.ceil(n4 / blocks)
        if per < loads * threads:
            continue          # the loads in flight would not all be issued
        if mode == 2 and loads * threads * 16 > 64 * 1024:
            continue
        outs = torch.empty(blocks, device=dev)
        us = timer.per_launch_us(
            lambda i: probe_read(bufs[i % pool], outs, threads, loads, mode, stream=stream), K)
        rows.append({"kind": "read", "mode": READ_MODES[mode], "blocks": blocks,
                     "threads": threads, "loads": loads, "us": round(us, 3),
                     "GBs": round(nbytes / us / 1e3, 1)})
        if plan:
            lab = f"read {READ_MODES[mode]} b{blocks} t{threads} l{loads}"
            plan.add(lab + " (warm)", kname[mode], K, bytes=nbytes)
            plan.add(lab, kname[mode], K, bytes=nbytes)
    reads = [r for r in rows if r["kind"] == "read"]
    best = min(reads, key=lambda r: r["us"])
    empty = min((r for r in rows if r["kind"] == "empty"), key=lambda r: r["us"])
    del bufs
    return {"bytes": nbytes, "launches_per_graph": K, "pool_buffers": pool, "rows": rows,
            "fastest_read": best, "fastest_empty": empty}


# ---------------------------------------------------------------------------
# Per-workgroup timeline
# ---------------------------------------------------------------------------

def timeline(torch, dev, xs, ys, NT: int, cfg: dict, launches: int = 64) -> Dict:
    """Back-to-back timeline launches of the fused kernel over the pool of
    pairs, and where each launch's time goes: workgroup dispatch ramp, first
    data back, last data back, the tail after it, and the gap to the next
    launch.  Stamps are the device wall clock (converted to µs)."""
    from . import _lib
    from .iqa import launch_workgroups, tiles_timeline
    N = xs[0].shape[0]
    pool = len(xs)
    nwg = launch_workgroups(N, NT, cfg)
    stream = torch.cuda.Stream(dev)
    stamps = torch.zeros(launches, nwg * 8, dtype=torch.int64, device=dev)
    ns = N // NT
    out = {"lisi": torch.empty(ns, ns, device=dev), "auglisi": torch.empty(ns, ns, device=dev)}
    for i in range(8):   # warm-up
        tiles_timeline(xs[i % pool], ys[i % pool], NT, cfg, stamps[0], stream=stream, out=out)
    torch.cuda.synchronize()
    timer = GraphTimer(torch, dev, stream)
    g = timer.capture(lambda i: tiles_timeline(xs[i % pool], ys[i % pool], NT, cfg, stamps[i],
                                               stream=stream, out=out), launches)
    ms = timer.replay_ms(g)[0]
    del g
    res = timeline_stats(stamps.view(launches, nwg, 8).cpu().numpy(),
                         int(_lib.load().iqa_wall_clock_khz()), ms * 1e3 / launches, 8 * N * N)
    return {"N": N, "NT": NT, "cfg": cfg, **res}


def read_timeline(torch, dev, nbytes: int, blocks: int, threads: int, loads: int,
                  launches: int = 64, pool_bytes: float = 1.0 * 2 ** 30) -> Dict:
    """The same timeline for the plain register read of `nbytes` per launch
    (the read floor's kernel), over distinct buffers."""
    from . import _lib
    from .iqa import probe_read_timeline
    stream = torch.cuda.Stream(dev)
    bufs = distinct_buffers(torch, dev, nbytes, pool_bytes)
    pool = len(bufs)
    stamps = torch.zeros(launches, blocks * 8, dtype=torch.int64, device=dev)
    outs = torch.empty(blocks, device=dev)
    for i in range(8):   # warm-up
        probe_read_timeline(bufs[i % pool], outs, threads, loads, stamps[0], stream=stream)
    torch.cuda.synchronize()
    timer = GraphTimer(torch, dev, stream)
    g = timer.capture(lambda i: probe_read_timeline(bufs[i % pool], outs, threads, loads,
                                                    stamps[i], stream=stream), launches)
    ms = timer.replay_ms(g)[0]
    del g
    res = timeline_stats(stamps.view(launches, blocks, 8).cpu().numpy(),
                         int(_lib.load().iqa_wall_clock_khz()), ms * 1e3 / launches, nbytes)
    del bufs
    return {"bytes": nbytes, "blocks": blocks, "threads": threads, "loads": loads, **res}


def timeline_stats(records, khz: int, event_us: float, bytes_launch: int) -> Dict:
    """Where each launch's time goes, from per-workgroup stamp records
    (launches x workgroups x 8: entry, first data, last data, exit, XCC_ID,
    HW_ID, index, split word): workgroup dispatch ramp, first data back, last
    data back, the tail after it, and the gap to the next launch (µs)."""
    st = np.asarray(records).astype(np.float64)
    launches, nwg = st.shape[0], st.shape[1]
    tick_us = 1e3 / khz
    entry, first, last, end = (st[:, :, k] for k in range(4))
    base = entry.min(axis=1, keepdims=True)
    ramp = (entry.max(axis=1) - entry.min(axis=1)) * tick_us
    first_lat = np.median(first - entry, axis=1) * tick_us
    data_end = (last.max(axis=1) - base[:, 0]) * tick_us
    tail = (end.max(axis=1) - last.max(axis=1)) * tick_us
    span = (end.max(axis=1) - base[:, 0]) * tick_us
    gaps = (entry.min(axis=1)[1:] - end.max(axis=1)[:-1]) * tick_us
    wg_busy = np.median(end - entry, axis=1) * tick_us
    xcc = st[0, :, 4].astype(np.int64) & 0xF
    per_xcd = np.bincount(xcc, minlength=8).tolist()
    fin = (st[:, :, 7].astype(np.int64) >> 32) == 1
    # a finishing workgroup's exit after its own last data, against the others'
    fin_tail = np.nanmedian(np.where(fin, end - last, np.nan), axis=1) * tick_us
    other_tail = np.nanmedian(np.where(~fin, end - last, np.nan), axis=1) * tick_us \
        if (~fin).any() else None

    def stat(a):
        a = np.asarray(a)
        return {"median": round(float(np.median(a)), 3), "min": round(float(a.min()), 3),
                "p90": round(float(np.percentile(a, 90)), 3)}

    span_med = float(np.median(span))
    return {
        "workgroups": nwg, "launches": launches, "wall_clock_khz": khz,
        "event_us_per_launch": round(event_us, 3),
        "dispatch_ramp_us": stat(ramp),
        "first_data_us": stat(first_lat),
        "last_data_us": stat(data_end),
        "tail_us": stat(tail),
        "span_us": stat(span),
        "gap_to_next_launch_us": stat(gaps) if gaps.size else None,
        "workgroup_busy_us": stat(wg_busy),
        "workgroups_per_xcd": per_xcd,
        "finishing_wg_exit_after_data_us": stat(fin_tail),
        "other_wg_exit_after_data_us": stat(other_tail) if other_tail is not None else None,
        "data_phase_GBs": round(bytes_launch / np.median(data_end) / 1e3, 1),
        "span_GBs": round(bytes_launch / span_med / 1e3, 1),
        "ideal_us_at_peak": round(bytes_launch / HBM_PEAK_GBS / 1e3, 3),
    }


# ---------------------------------------------------------------------------
# rocprofv3 kernel-trace summaries
# ---------------------------------------------------------------------------

def trace_summary(trace_csv: str, plan_json: str) -> List[dict]:
    """Match a rocprofv3 kernel trace (CSV) to a launch plan: walk the
    dispatches in start order and give each segment the next `count`
    dispatches whose kernel name contains the segment's kernel; other
    dispatches (fills, copies) are skipped.  Per segment: mean, median, min,
    p90 of the kernel durations (ns)."""
    import csv
    with open(plan_json) as fh:
        segs = json.load(fh)["segments"]
    rows = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    out, i = [], 0
    for seg in segs:
        durs = []
        while len(durs) < seg["count"] and i < len(rows):
            s, e, name = rows[i]
            i += 1
            if seg["kernel"] in name:
                durs.append(e - s)
        d = np.array(durs, dtype=np.float64)
        rec = {k: v for k, v in seg.items() if k != "count"}
        rec.update({"dispatches": int(d.size), "expected": seg["count"]})
        if d.size:
            rec.update({"mean_ns": float(d.mean()), "median_ns": float(np.median(d)),
                        "min_ns": float(d.min()), "p90_ns": float(np.percentile(d, 90))})
        out.append(rec)
    return out


# ---------------------------------------------------------------------------
# HBM traffic from rocprofv3 counters
# ---------------------------------------------------------------------------

CALIBRATION_KERNEL = "copyBuffer"     # the runtime's device-to-device copy
CALIBRATION_BYTES = 256 << 20         # bench.py --profile copies 256 MiB, 3 times


def _counter_rows(path: str, kernel: str) -> List[float]:
    import csv
    with open(path) as fh:
        return [float(r["Counter_Value"]) for r in csv.DictReader(fh) if kernel in r["Kernel_Name"]]


def traffic(fetch_csv: str, write_csv: str, kernel: str, algorithmic_bytes: int) -> Dict:
    """HBM bytes per launch of `kernel` from one FETCH_SIZE and one WRITE_SIZE
    counter pass (KiB per dispatch), each scaled by what the same counter
    reads for the run's 256 MiB device copies (the largest copyBuffer
    dispatches): bytes = KiB * 1024 * (copy bytes / copy KiB counted)."""
    out = {}
    for name, path, copy_kib_true in (("fetch", fetch_csv, CALIBRATION_BYTES / 1024),
                                      ("write", write_csv, CALIBRATION_BYTES / 1024)):
        k = _counter_rows(path, kernel)
        cal = sorted(_counter_rows(path, CALIBRATION_KERNEL))[-3:]
        if not k or not cal:
            raise ValueError(f"{path}: no {kernel} or calibration dispatches")
        scale = copy_kib_true / (sum(cal) / len(cal))
        out[f"{name}_kib_per_dispatch"] = round(sum(k) / len(k), 2)
        out[f"{name}_dispatches"] = len(k)
        out[f"{name}_scale"] = round(scale, 4)
    hbm = (out["fetch_kib_per_dispatch"] * out["fetch_scale"] +
           out["write_kib_per_dispatch"] * out["write_scale"]) * 1024
    out["hbm_bytes_per_launch"] = int(round(hbm))
    out["algorithmic_bytes_per_launch"] = int(algorithmic_bytes)
    out["ratio"] = round(hbm / algorithmic_bytes, 5)
    return out


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="Summarise a rocprofv3 kernel trace against a "
                                             "launch plan written by bench.py, or turn two "
                                             "counter passes into HBM bytes per launch")
    ap.add_argument("--trace", help="rocprofv3 *_kernel_trace.csv")
    ap.add_argument("--plan", help="plan JSON written by bench.py --plan-out")
    ap.add_argument("--all", action="store_true", help="also list the untimed (warm) segments")
    ap.add_argument("--fetch", help="FETCH_SIZE *_counter_collection.csv")
    ap.add_argument("--write", help="WRITE_SIZE *_counter_collection.csv")
    ap.add_argument("--kernel", default="tiles_kernel")
    ap.add_argument("--algorithmic-bytes", type=int, default=0)
    args = ap.parse_args(argv)
    if args.fetch:
        print(json.dumps(traffic(args.fetch, args.write, args.kernel, args.algorithmic_bytes),
                         indent=1))
        return 0
    recs = trace_summary(args.trace, args.plan)
    print("| segment | dispatches | median ns | min ns | p90 ns | mean ns | GB/s (median) "
          "| % of 8 TB/s |")
    print("|---|---|---|---|---|---|---|---|")
    for r in recs:
        if r["label"].endswith("(warm)") and not args.all:
            continue
        if "median_ns" not in r:
            print(f"| {r['label']} | {r['dispatches']}/{r['expected']} | - | - | - | - | - | - |")
            continue
        b = r.get("bytes")
        gbs = f"{b / r['median_ns']:.1f}" if b else "-"
        pct = f"{100 * b / r['median_ns'] / HBM_PEAK_GBS:.1f}" if b else "-"
        print(f"| {r['label']} | {r['dispatches']}/{r['expected']} | {r['median_ns']:.0f} | "
              f"{r['min_ns']:.0f} | {r['p90_ns']:.0f} | {r['mean_ns']:.0f} | {gbs} | {pct} |")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
