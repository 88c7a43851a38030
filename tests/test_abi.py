"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/iqa.h declares, and rejects bad arguments before any HIP call."""

from __future__ import annotations

import ctypes
import math
import os
import re
import subprocess
import sys

import pytest

from paper_2501_10653_amd import _lib
from paper_2501_10653_amd._lib import LaunchCfg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iqa.h")

OK, NULL, SHAPE, ALIGN, PARAM, HIP, CONFIG, CAPTURE, BUDGET, TIMEOUT, SCRATCH = range(11)
FAKE = 1 << 20          # 16-byte-aligned stand-in for a device pointer (never dereferenced)
C6 = 1e-6


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[a-z_ *]*?\b([a-z_]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("iqa_tiles", "lisi_tiles", "auglisi_tiles", "iqa_status_str"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(declared_functions()) <= exported


def test_status_strings():
    lib = _lib.load()
    for s in range(11):
        assert lib.iqa_status_str(s).decode().startswith(_lib.STATUS_NAMES[s])
    assert b"unknown" in lib.iqa_status_str(99)
    assert lib.iqa_version() >= 100


def call_tiles(x=FAKE, y=FAKE, N=2048, NT=64, D=C6 / 2, C1=C6, C2=C6, C=C6, lisi=FAKE,
               aug=FAKE, sums=None):
    return _lib.load().iqa_tiles(x, y, N, NT, D, C1, C2, C, lisi, aug, sums, None)


@pytest.mark.parametrize("kw,status", [
    (dict(x=None), NULL), (dict(y=None), NULL), (dict(lisi=None, aug=None), NULL),
    (dict(N=0), SHAPE), (dict(NT=0), SHAPE), (dict(N=-4, NT=2), SHAPE), (dict(N=100, NT=7), SHAPE),
    (dict(N=64, NT=128), SHAPE), (dict(N=(1 << 17) + 2, NT=2), SHAPE),
    (dict(x=FAKE + 2), ALIGN), (dict(lisi=FAKE + 1), ALIGN), (dict(sums=FAKE + 4), ALIGN),
    (dict(C1=0.0), PARAM), (dict(C2=-1.0), PARAM), (dict(C=float("nan")), PARAM),
    (dict(D=float("inf")), PARAM), (dict(C1=1e-40), PARAM), (dict(D=0.0), PARAM),
])
def test_validation_before_launch(kw, status):
    assert call_tiles(**kw) == status


def test_split_entry_points_validate_only_their_constants():
    lib = _lib.load()
    # lisi_tiles ignores C, auglisi_tiles ignores D, C1, C2: only their own are checked
    assert lib.lisi_tiles(FAKE, FAKE, 64, 8, 0.5, 0.0, C6, FAKE, None) == PARAM
    assert lib.lisi_tiles(FAKE, FAKE, 64, 8, 0.5, C6, C6, None, None) == NULL
    assert lib.auglisi_tiles(FAKE, FAKE, 64, 8, 0.0, FAKE, None) == PARAM
    assert lib.auglisi_tiles(FAKE, None, 64, 8, C6, FAKE, None) == NULL
    assert lib.auglisi_tiles(FAKE, FAKE, 64, 7, C6, FAKE, None) == SHAPE


def default_cfg(N, NT, x=FAKE, y=FAKE):
    c = LaunchCfg()
    st = _lib.load().iqa_default_cfg(N, NT, x, y, ctypes.byref(c))
    return st, c.as_dict()


@pytest.mark.parametrize("N,NT", [(256, 32), (2048, 64), (1024, 256), (8192, 16), (4096, 128),
                                  (12, 3), (10, 10), (300, 12), (1000, 8), (7, 1), (1, 1),
                                  (512, 512), (8192, 8192), (6, 2)])
def test_default_cfg_is_valid(N, NT):
    st, c = default_cfg(N, NT)
    assert st == OK
    assert NT % c["vec"] == 0
    assert _lib.load().iqa_check_cfg(N, NT, ctypes.byref(LaunchCfg.from_dict(c))) == OK


def test_default_cfg_follows_alignment():
    assert default_cfg(64, 8, FAKE + 8, FAKE)[1]["vec"] == 2
    assert default_cfg(64, 8, FAKE + 4, FAKE)[1]["vec"] == 1
    assert default_cfg(66, 6, FAKE, FAKE)[1]["vec"] == 2
    assert default_cfg(63, 9, FAKE, FAKE)[1]["vec"] == 1
    assert default_cfg(64, 9)[0] == SHAPE


@pytest.mark.parametrize("bad", [
    dict(vec=3), dict(vec=4, waves=3), dict(waves=16, unroll=8), dict(waves=32), dict(seg=12), dict(seg=128), dict(rp=3),
    dict(seg=16, rp=8), dict(ksplit=0), dict(ksplit=3), dict(vec=2, waves=2),
    dict(vec=1, unroll=8), dict(unroll=16), dict(unroll=2), dict(waves=8, ksplit=16),
])
def test_check_cfg_rejects(bad):
    base = dict(vec=4, waves=1, unroll=8, seg=16, rp=4, ksplit=1)
    base.update(bad)
    st = _lib.load().iqa_check_cfg(2048, 64, ctypes.byref(LaunchCfg.from_dict(base)))
    assert st == CONFIG


def test_cfg_call_rejects_invalid_config_before_launch():
    bad = LaunchCfg.from_dict(dict(vec=4, waves=5, unroll=4, seg=16, rp=1, ksplit=1))
    st = _lib.load().iqa_tiles_cfg(FAKE, FAKE, 2048, 64, C6 / 2, C6, C6, C6, FAKE, None, None,
                                   ctypes.byref(bad), None)
    assert st == CONFIG


def make_pairs(n, **over):
    arr = (_lib.IqaPair * n)()
    for i in range(n):
        kw = dict(x=FAKE, y=FAKE, N=256, NT=32, D=C6 / 2, C1=C6, C2=C6, C=C6, lisi=FAKE,
                  auglisi=FAKE, sums=None)
        kw.update(over)
        arr[i] = _lib.IqaPair(**kw)
    return arr


@pytest.mark.parametrize("over,status", [
    (dict(), OK), (dict(NT=30, N=300), CONFIG), (dict(x=FAKE + 4), ALIGN), (dict(N=100, NT=8), SHAPE),
    (dict(C=0.0), PARAM), (dict(lisi=None, auglisi=None), NULL), (dict(y=None), NULL),
])
def test_batch_describe_validates_every_pair(over, status):
    import numpy as np
    arr = make_pairs(3, **over)
    buf = np.zeros(3 * _lib.BATCH_DESC_BYTES, np.uint8)
    units = ctypes.c_int64(-1)
    st = _lib.load().iqa_batch_describe(arr, 3, buf.ctypes.data, ctypes.byref(units))
    assert st == status
    if status == OK:
        # tile groups: 8 rows of tiles x ceil(8 / tiles-per-wave); a unit is
        # four groups (one wave each) or one group (four waves splitting rows)
        c = LaunchCfg()
        assert _lib.load().iqa_batch_cfg(256, 32, ctypes.byref(c)) == OK
        ht = 64 // (c.seg * c.rp)
        groups = 8 * -(-8 // ht)
        assert units.value == 3 * (groups if c.waves == 4 else -(-groups // 4))


def test_batch_launch_validation():
    lib = _lib.load()
    assert lib.iqa_tiles_batched(None, 1, 1, 2048, None) == NULL
    assert lib.iqa_tiles_batched(FAKE, 0, 1, 2048, None) == SHAPE
    assert lib.iqa_tiles_batched(FAKE, 1, 0, 2048, None) == SHAPE
    assert lib.iqa_tiles_batched(FAKE, 1, 1, 2046, None) == CONFIG
    assert lib.iqa_tiles_batched(FAKE + 8, 1, 1, 2048, None) == ALIGN


def test_inline_batch_launch_validation():
    """Descriptors by value: at most IQA_BATCH_INLINE_MAX pairs, checked
    before anything is copied or launched."""
    import numpy as np
    lib = _lib.load()
    host = np.zeros(17 * _lib.BATCH_DESC_BYTES, np.uint8)
    p = host.ctypes.data
    assert lib.iqa_tiles_batched_inline(None, 1, 1, 2048, None) == NULL
    assert lib.iqa_tiles_batched_inline(p, 0, 1, 2048, None) == SHAPE
    assert lib.iqa_tiles_batched_inline(p, _lib.BATCH_INLINE_MAX + 1, 1, 2048, None) == SHAPE
    assert lib.iqa_tiles_batched_inline(p, 1, 0, 2048, None) == SHAPE
    assert lib.iqa_tiles_batched_inline(p, 1, 1, 2046, None) == CONFIG
    header = open(os.path.join(ROOT, "include", "iqa.h")).read()
    assert f"#define IQA_BATCH_INLINE_MAX {_lib.BATCH_INLINE_MAX}" in header


def test_inline_batch_checks_the_unit_numbering():
    """The inline launch holds the descriptors on the host, so a unit count
    or pair order that does not match what iqa_batch_describe wrote is refused
    before anything is launched."""
    import numpy as np
    lib = _lib.load()
    arr = make_pairs(3)
    buf = np.zeros(3 * _lib.BATCH_DESC_BYTES, np.uint8)
    units = ctypes.c_int64(-1)
    assert lib.iqa_batch_describe(arr, 3, buf.ctypes.data, ctypes.byref(units)) == OK
    u = units.value
    for count, total in ((3, u + 1), (3, u - 1), (2, u), (3, 2 * u)):
        assert lib.iqa_tiles_batched_inline(buf.ctypes.data, count, total, 2048, None) == CONFIG
    swapped = buf.copy().reshape(3, -1)
    swapped[[0, 1]] = swapped[[1, 0]]
    # pairs 0 and 1 have the same geometry, so swapping them keeps the sum but
    # not the numbering: pair 0 then claims to start at pair 1's first unit
    assert lib.iqa_tiles_batched_inline(swapped.ctypes.data, 3, u, 2048, None) == CONFIG


def test_batch_units_follow_each_pairs_geometry():
    """A unit is one workgroup: four tile groups of a one-wave pair, one tile
    group of a four-wave pair.  Described totals follow each pair's geometry,
    and the inline launch accepts exactly that total."""
    import numpy as np
    lib = _lib.load()
    lib.iqa_tune_clear()
    try:
        one = LaunchCfg.from_dict(dict(vec=4, waves=1, unroll=8, seg=8, rp=2, ksplit=1))
        four = LaunchCfg.from_dict(dict(vec=4, waves=4, unroll=8, seg=8, rp=2, ksplit=1))
        assert lib.iqa_tune_set(256, 32, _lib.TUNE_BATCH, ctypes.byref(one)) == OK
        assert lib.iqa_tune_set(512, 32, _lib.TUNE_BATCH, ctypes.byref(four)) == OK
        arr = (_lib.IqaPair * 3)()
        for i, N in enumerate((256, 512, 256)):
            arr[i] = _lib.IqaPair(FAKE, FAKE, N, 32, C6 / 2, C6, C6, C6, FAKE, FAKE, None)
        buf = np.zeros(3 * _lib.BATCH_DESC_BYTES, np.uint8)
        units = ctypes.c_int64(-1)
        assert lib.iqa_batch_describe(arr, 3, buf.ctypes.data, ctypes.byref(units)) == OK
        # seg 8, rp 2: 4 tiles per wave.  256/32: 8 x 2 groups -> 4 units;
        # 512/32: 16 x 4 groups, each its own unit -> 64 units
        assert units.value == 4 + 64 + 4
        begins = [int(np.frombuffer(buf[i * 128 + 120:i * 128 + 128].tobytes(), np.int64)[0])
                  for i in range(3)]
        assert begins == [0, 4, 68]
        for total in (units.value - 1, units.value + 1):
            assert lib.iqa_tiles_batched_inline(buf.ctypes.data, 3, total, 2048, None) == CONFIG
    finally:
        lib.iqa_tune_clear()


def test_tune_registry():
    lib = _lib.load()
    lib.iqa_tune_clear()
    baseline = default_cfg(2048, 64)[1]
    try:
        good = LaunchCfg.from_dict(dict(vec=4, waves=1, unroll=8, seg=16, rp=2, ksplit=1))
        assert lib.iqa_tune_set(2048, 64, _lib.TUNE_SINGLE, ctypes.byref(good)) == OK
        st, c = default_cfg(2048, 64)
        assert st == OK and c == good.as_dict()
        # unaligned images ignore tuned vec-4 entries
        assert default_cfg(2048, 64, FAKE + 4, FAKE)[1]["vec"] == 1
        assert lib.iqa_tune_set(2048, 64, _lib.TUNE_BATCH, ctypes.byref(good)) == OK
        c2 = LaunchCfg()
        assert lib.iqa_batch_cfg(2048, 64, ctypes.byref(c2)) == OK and c2.as_dict() == good.as_dict()
        # N == 0 registers for every N with this NT
        wide = LaunchCfg.from_dict(dict(vec=4, waves=1, unroll=8, seg=16, rp=4, ksplit=1))
        assert lib.iqa_tune_set(0, 64, _lib.TUNE_BATCH, ctypes.byref(wide)) == OK
        assert lib.iqa_batch_cfg(4096, 64, ctypes.byref(c2)) == OK and c2.as_dict() == wide.as_dict()
        # the server's geometry: its own entries, else the batch geometry
        c3 = LaunchCfg()
        assert lib.iqa_serve_cfg(8192, 64, ctypes.byref(c3)) == OK and c3.as_dict() == wide.as_dict()
        coop = LaunchCfg.from_dict(dict(vec=4, waves=4, unroll=8, seg=16, rp=2, ksplit=1))
        assert lib.iqa_tune_set(1024, 64, _lib.TUNE_SERVE, ctypes.byref(coop)) == OK
        assert lib.iqa_serve_cfg(1024, 64, ctypes.byref(c3)) == OK and c3.as_dict() == coop.as_dict()
        assert lib.iqa_batch_cfg(1024, 64, ctypes.byref(c2)) == OK and c2.as_dict() == wide.as_dict()
        assert lib.iqa_serve_cfg(1024, 62, ctypes.byref(c3)) == SHAPE
        assert lib.iqa_serve_cfg(1000, 20, ctypes.byref(c3)) == OK
        bad = LaunchCfg.from_dict(dict(vec=4, waves=2, unroll=8, seg=16, rp=2, ksplit=1))
        assert lib.iqa_tune_set(2048, 64, _lib.TUNE_BATCH, ctypes.byref(bad)) == CONFIG
        assert lib.iqa_tune_set(2048, 64, _lib.TUNE_SERVE, ctypes.byref(bad)) == CONFIG
        assert lib.iqa_tune_set(2048, 64, 7, ctypes.byref(good)) == CONFIG
        assert lib.iqa_tune_set(2048, 63, 0, ctypes.byref(good)) == SHAPE
    finally:
        lib.iqa_tune_clear()
    assert default_cfg(2048, 64)[1] == baseline
    assert lib.iqa_batch_default_waves() >= 4


@pytest.mark.parametrize("over", [dict(streams=0), dict(streams=17), dict(max_batch=0),
                                  dict(hbm_budget_bytes=0), dict(waves=6), dict(host_arena_bytes=-1),
                                  dict(idle_spin_ns=-1), dict(idle_spin_ns=2_000_000_000)])
def test_server_options_validated_before_any_gpu_call(over):
    kw = dict(hbm_budget_bytes=1 << 30, host_arena_bytes=0, waves=0, streams=2, max_batch=64,
              D=C6 / 2, C1=C6, C2=C6, C=C6)
    kw.update(over)
    opts = _lib.ServerOpts(**kw)
    h = ctypes.c_void_p()
    assert _lib.load().iqa_server_create(ctypes.byref(opts), ctypes.byref(h)) == CONFIG
    assert not h.value


def test_header_is_plain_c_and_links(tmp_path):
    """A C program built with gcc against include/iqa.h links to the library
    and gets the documented statuses back."""
    exe = tmp_path / "c_abi_check"
    src = os.path.join(ROOT, "tests", "c_abi_check.c")
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    src, "-o", str(exe), "-L", libdir, "-l:libiqa_hip.so",
                    f"-Wl,-rpath,{libdir}"], check=True, capture_output=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    sizes = [int(v) for v in res.stdout.split("sizes")[1].split("\n")[0].split()]
    mirrors = [LaunchCfg, _lib.IqaPair, _lib.ServerOpts, _lib.Request, _lib.Completion,
               _lib.ServerStats]
    assert sizes == [ctypes.sizeof(m) for m in mirrors]


def test_missing_library_fails_loudly(tmp_path):
    """No CPU fallback: without the built library every entry point raises."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2501_10653_amd import _lib\n"
            "_lib.LIB_PATH = %r\n"
            "try:\n"
            "    _lib.load()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(1)\n") % (ROOT, str(tmp_path / "missing.so"))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert res.returncode == 0 and "not built" in res.stdout


def test_noalloc_refuses_shapes_beyond_its_scratch_before_any_hip_call():
    """A split shape whose partial sums exceed the fixed scratch array is
    refused with IQA_ERR_SCRATCH, and validation errors come first, as for
    iqa_tiles_cfg."""
    lib = _lib.load()
    big = LaunchCfg.from_dict(dict(vec=4, waves=1, unroll=4, seg=64, rp=1, ksplit=64))
    # 65536^2 / 2048: 1024 tile groups x 64 parts x 16 B = 1 MiB of partials
    assert lib.iqa_tiles_noalloc(FAKE, FAKE, 65536, 2048, C6 / 2, C6, C6, C6, FAKE, FAKE, None,
                                 ctypes.byref(big), None) == SCRATCH
    assert lib.iqa_tiles_noalloc(None, FAKE, 65536, 2048, C6 / 2, C6, C6, C6, FAKE, FAKE, None,
                                 ctypes.byref(big), None) == NULL
    assert lib.iqa_tiles_noalloc(FAKE, FAKE, 65536, 2047, C6 / 2, C6, C6, C6, FAKE, FAKE, None,
                                 None, None) == SHAPE
    assert lib.iqa_tiles_noalloc(FAKE, FAKE, 2048, 64, C6 / 2, 0.0, C6, C6, FAKE, FAKE, None,
                                 None, None) == PARAM
