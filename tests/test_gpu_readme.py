"""The usage example in README.md runs as written, and its served result is
bitwise the single-pair launch with the batch geometry."""

from __future__ import annotations

import os
import re

import pytest
import torch

from tests.gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    from paper_2501_10653_amd import iqa_tiles
    from paper_2501_10653_amd.serve import serve_cfg
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"```python\n(.*?)```", text, re.S).group(1)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    assert tuple(ns["res"].lisi.shape) == (32, 32) and tuple(ns["res"].sums.shape) == (1024, 4)
    assert [lv.lisi.shape[0] for lv in ns["levels"]] == [32, 16, 8, 4, 2, 1]
    assert len(ns["b"].results) == 2 and tuple(ns["b"].results[1].lisi.shape) == (32, 32)
    done = ns["done"]
    assert len(done) == 1 and done[0]["status"] == 0
    req, x, y = ns["req"], ns["x"], ns["y"]
    single = iqa_tiles(y, x, 64, cfg=serve_cfg(2048, 64))
    torch.cuda.synchronize()
    assert torch.equal(req.lisi.view(torch.int32), single.lisi.view(torch.int32))
    assert torch.equal(req.auglisi.view(torch.int32), single.auglisi.view(torch.int32))
