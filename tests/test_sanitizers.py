"""The library's host code under sanitizers (CPU only, no GPU).

The HIP sources are compiled with ThreadSanitizer, or with AddressSanitizer
and UndefinedBehaviorSanitizer, on their host side only (the gfx950 code is
built as usual and never launched here), and linked into two plain-C
drivers:

* tests/c_server_stress.c: two threads submit requests to a dry-run server
  (the real scheduler, no GPU) while a third polls completions; then drain
  and destroy.
* tests/c_abi_check.c: the entry points' argument validation.

Any sanitizer report fails the test.  Builds are cached under _build/ by a
digest of the sources and flags."""

import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_10653_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SOURCES = [os.path.join(CSRC, f) for f in ("iqa_server.hip", "iqa_kernels.hip")]
SANITIZERS = {"tsan": ["thread"], "asan": ["address", "undefined"]}

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and shutil.which("gcc")),
                                reason="needs hipcc and gcc")


def _digest(paths, extra) -> str:
    h = hashlib.sha256(" ".join(extra).encode())
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    for inc in ("iqa_internal.h", "tuned_table.inc"):
        with open(os.path.join(CSRC, inc), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "iqa.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _build(kind: str, driver: str) -> str:
    san = SANITIZERS[kind]
    host_san = [a for s in san for a in ("-Xarch_host", f"-fsanitize={s}")]
    lib_dir = os.path.join(ROOT, "_build", "sanitizers", f"{kind}-{_digest(SOURCES, san)}")
    os.makedirs(lib_dir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(lib_dir, os.path.basename(src) + ".o")
        if not os.path.exists(obj):
            subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                            *host_san, "-fno-omit-frame-pointer",
                            "-Wno-unused-command-line-argument", "-I",
                            os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o",
                            obj + ".tmp"], check=True, capture_output=True)
            os.replace(obj + ".tmp", obj)
        return obj

    with ThreadPoolExecutor(len(SOURCES)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    drv = os.path.join(ROOT, "tests", driver + ".c")
    exe = os.path.join(lib_dir, f"{driver}-{_digest([drv], san)}")
    if os.path.exists(exe):
        return exe
    dobj = exe + ".o"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-Werror",
                    f"-fsanitize={','.join(san)}", "-fno-omit-frame-pointer",
                    "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-c", drv, "-o", dobj], check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950", *host_san, dobj, *objs, "-o", exe + ".tmp",
                    "-lpthread"], check=True, capture_output=True)
    os.replace(exe + ".tmp", exe)
    return exe


def _run(exe: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=67:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=68")
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)


def _clean(r: subprocess.CompletedProcess, ok_line: str) -> None:
    reports = [l for l in r.stderr.splitlines()
               if "ThreadSanitizer" in l or "AddressSanitizer" in l or "runtime error" in l]
    assert r.returncode == 0 and not reports, (r.returncode, "\n".join(reports[:20]),
                                                r.stderr[-4000:])
    assert ok_line in r.stdout


def test_server_scheduler_under_threadsanitizer():
    _clean(_run(_build("tsan", "c_server_stress")), "stress ok")


def test_server_scheduler_under_asan_and_ubsan():
    _clean(_run(_build("asan", "c_server_stress")), "stress ok")


def test_argument_validation_under_asan_and_ubsan():
    _clean(_run(_build("asan", "c_abi_check")), "c_abi_check ok")
