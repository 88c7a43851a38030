"""Per-workload error of the FP32 kernel against the FP64 oracle.

Asserts the contract (LISI and sums: relative error <= 1e-5 per tile; augLISI:
|g - o| <= 1e-5 * max(|o|, P/(Sx+Sy+C))) and, when IQA_PRECISION_REPORT names
a file, writes the statistics there as JSON (max and median plain relative
error per output, tiles in the r > 0.5 regime).
"""

from __future__ import annotations

import json
import os

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import iqa_tiles, synth
from tests.gpu_util import aug_errors, oracle_for, rel_errors, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

OUT = os.environ.get("IQA_PRECISION_REPORT")

WORKLOADS = [("small 256/32", synth.spec_small()), ("paper 2048/64", synth.spec_paper_shape())] + \
    [(f"sweep {N}/{NT}", synth.spec_sweep(N, NT)) for N in (1024, 2048, 4096, 8192)
     for NT in (16, 32, 64, 128, 256)] + \
    [("bright transient amp 2, 2048/64", (lambda: synth.bright_transient_pair(2048, 64, amp=2.0), 64)),
     ("bright transient amp 8, 2048/16", (lambda: synth.bright_transient_pair(2048, 16, amp=8.0), 16))]


def stats(g, o):
    e = rel_errors(g, o)
    return {"max": float(e.max()), "median": float(np.median(e))}


def test_precision_report():
    report = []
    for name, spec in WORKLOADS:
        if isinstance(spec, tuple):
            x, y, _ = spec[0]()
            NT = spec[1]
        else:
            x, y, _ = synth.make_pair(spec)
            NT = spec.NT
        res = iqa_tiles(to_dev(x), to_dev(y), NT, sums=True)
        torch.cuda.synchronize()
        ol, oa, osum = oracle_for(x, y, NT)
        gl = res.lisi.cpu().numpy().ravel()
        ga = res.auglisi.cpu().numpy().ravel()
        gs = res.sums.cpu().numpy()
        r = 1.0 - oa.ravel()
        row = {"workload": name, "tiles": int(gl.size),
               "lisi": stats(gl, ol.ravel()),
               "auglisi_plain": stats(ga, oa.ravel()),
               "auglisi_conditioned_max": float(aug_errors(ga, oa.ravel()).max()),
               "tiles_r_gt_half": int((r > 0.5).sum()),
               "sums_max": {k: float(rel_errors(gs[:, i], osum[:, i]).max())
                            for i, k in enumerate(("A", "P", "Sx", "Sy"))}}
        report.append(row)
        assert row["lisi"]["max"] <= 1e-5, name
        assert row["auglisi_conditioned_max"] <= 1e-5, name
        assert max(row["sums_max"].values()) <= 1e-5, name
    if OUT:
        with open(OUT, "w") as fh:
            json.dump(report, fh, indent=1)
    worst = max(r["lisi"]["max"] for r in report)
    print(f"worst LISI rel err {worst:.3g}")
