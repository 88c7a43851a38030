"""The library driven from plain C, with no Python or torch in the process:
tests/c_gpu_driver.c (hipMalloc, a HIP stream and the tile entry points) and
tests/c_server_driver.c (the serving entry points), checked against the
oracle on every tile."""

from __future__ import annotations

import os
import subprocess
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from paper_2501_10653_amd import synth
from tests.gpu_util import assert_parity, oracle_for, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "c_gpu_driver")
SERVER_DRIVER = os.path.join(ROOT, "tests", "c_server_driver")
IQA_ERR_ALIGN = 3


def _cases():
    rng = np.random.default_rng(31)
    x0, y0, _ = synth.make_pair(synth.spec_small())
    x1, y1 = synth.random_pair(1024, rng, neg_frac=0.3, nan_frac=0.01, scale=1.5)
    x2, y2, _ = synth.make_pair(synth.spec_paper_shape())
    return [("small 256/32", x0, y0, 32), ("random 1024/32", x1, y1, 32),
            ("paper 2048/64", x2, y2, 64)]


@pytest.mark.parametrize("case", range(3))
def test_c_driver_matches_oracle(case, tmp_path):
    assert os.path.exists(DRIVER), "tests/c_gpu_driver is not built: run __graft_entry__.build()"
    name, x, y, NT = _cases()[case]
    N = x.shape[0]
    ns = N // NT
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as fh:
        fh.write(np.array([N, NT], np.int64).tobytes())
        fh.write(np.ascontiguousarray(x, np.float32).tobytes())
        fh.write(np.ascontiguousarray(y, np.float32).tobytes())
    print(f"c driver: {name}", flush=True)
    res = subprocess.run([DRIVER, str(src), str(dst)], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    raw = np.fromfile(dst, dtype=np.int32, count=5)
    assert list(raw[:3]) == [0, 0, 0], raw
    assert raw[3] == IQA_ERR_ALIGN, raw
    assert raw[4] == 1, "lisi_tiles / auglisi_tiles differ from the fused entry point"
    vals = np.fromfile(dst, dtype=np.float32, offset=20)
    assert vals.size == 6 * ns * ns
    out = SimpleNamespace(lisi=torch.from_numpy(vals[:ns * ns].reshape(ns, ns).copy()),
                          auglisi=torch.from_numpy(vals[ns * ns:2 * ns * ns].reshape(ns, ns).copy()),
                          sums=torch.from_numpy(vals[2 * ns * ns:].reshape(ns * ns, 4).copy()))
    assert_parity(out, oracle_for(x, y, NT), what=name)


@pytest.mark.parametrize("N,NT", [(512, 32), (1024, 64)])
def test_c_server_driver_matches_single_launches_and_oracle(N, NT, tmp_path):
    assert os.path.exists(SERVER_DRIVER), \
        "tests/c_server_driver is not built: run __graft_entry__.build()"
    spec = synth.serving_references(count=1, Ns=(N,), seed=13)[0]
    ref, _, _ = synth.make_pair(spec)
    snaps = [synth.make_snapshot(spec, k) for k in range(6)]
    ns = N // NT
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as fh:
        fh.write(np.array([N, NT, len(snaps)], np.int64).tobytes())
        fh.write(np.ascontiguousarray(ref, np.float32).tobytes())
        for s in snaps:
            fh.write(np.ascontiguousarray(s, np.float32).tobytes())
    print(f"c server driver: {N}/{NT}, {len(snaps)} requests", flush=True)
    res = subprocess.run([SERVER_DRIVER, str(src), str(dst)], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    st = np.fromfile(dst, dtype=np.int32, count=7)
    assert list(st[:4]) == [0, 0, 0, 0], st          # create, add_reference, submit, drain
    assert st[4] == len(snaps) and st[5] == 1, st     # every completion polled, all OK
    assert st[6] == 1, "served results differ from the single-pair launches"
    vals = np.fromfile(dst, dtype=np.float32, offset=28).reshape(2, len(snaps), ns, ns)
    for k, s in enumerate(snaps):
        out = SimpleNamespace(lisi=torch.from_numpy(vals[0, k].copy()),
                              auglisi=torch.from_numpy(vals[1, k].copy()), sums=None)
        assert_parity(out, oracle_for(s, ref, NT), what=f"request {k}")
