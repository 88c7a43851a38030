"""ctypes loader for the HIP library ``libiqa_hip.so`` (C ABI of include/iqa.h).

The library is required: if it is missing or fails to load, every entry point
raises.  There is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libiqa_hip.so")

IQA_OK = 0
STATUS_NAMES = {
    0: "IQA_OK", 1: "IQA_ERR_NULL", 2: "IQA_ERR_SHAPE", 3: "IQA_ERR_ALIGN",
    4: "IQA_ERR_PARAM", 5: "IQA_ERR_HIP", 6: "IQA_ERR_CONFIG", 7: "IQA_ERR_CAPTURE",
    8: "IQA_ERR_BUDGET", 9: "IQA_ERR_TIMEOUT", 10: "IQA_ERR_SCRATCH",
}


class LaunchCfg(ctypes.Structure):
    """Mirror of ``iqa_launch_cfg``."""

    _fields_ = [("vec", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("seg", ctypes.c_int32),
                ("rp", ctypes.c_int32), ("ksplit", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def from_dict(cls, d: dict) -> "LaunchCfg":
        return cls(**{k: int(d[k]) for k, _ in cls._fields_})


class IqaPair(ctypes.Structure):
    """Mirror of ``iqa_pair``."""

    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("NT", ctypes.c_int64), ("D", ctypes.c_float), ("C1", ctypes.c_float),
                ("C2", ctypes.c_float), ("C", ctypes.c_float), ("lisi", ctypes.c_void_p),
                ("auglisi", ctypes.c_void_p), ("sums", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    """Mirror of ``iqa_server_opts``."""

    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("host_arena_bytes", ctypes.c_int64),
                ("waves", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("D", ctypes.c_float), ("C1", ctypes.c_float),
                ("C2", ctypes.c_float), ("C", ctypes.c_float), ("idle_spin_ns", ctypes.c_int64)]


class Request(ctypes.Structure):
    """Mirror of ``iqa_request``."""

    _fields_ = [("snapshot_dev", ctypes.c_void_p), ("snapshot_host", ctypes.c_void_p),
                ("lisi", ctypes.c_void_p), ("auglisi", ctypes.c_void_p),
                ("sums", ctypes.c_void_p), ("NT", ctypes.c_int64), ("ref_id", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tag", ctypes.c_uint64),
                ("ready_event", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    """Mirror of ``iqa_completion``."""

    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("t_poll_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    """Mirror of ``iqa_server_stats``."""

    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_batch", ctypes.c_int64), ("in_flight_bytes", ctypes.c_int64),
                ("peak_in_flight_bytes", ctypes.c_int64), ("last_hip_error", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


BATCH_DESC_BYTES = 128
BATCH_INLINE_MAX = 16
TUNE_SINGLE = 0
TUNE_BATCH = 1
TUNE_SERVE = 2
NOALLOC_SCRATCH_BYTES = 1 << 20
PROBE_READ_REGS = 0
PROBE_READ_REGS_STRUCT = 1
PROBE_READ_LDS = 2


class IqaError(RuntimeError):
    def __init__(self, status: int, where: str, hip_error: int = 0):
        self.status = status
        self.hip_error = hip_error
        msg = _status_str(status)
        if hip_error:
            msg += f" (hip error {hip_error})"
        super().__init__(f"{where}: {msg}")


_lib: Optional[ctypes.CDLL] = None


def _status_str(status: int) -> str:
    try:
        return load().iqa_status_str(status).decode()
    except Exception:  # noqa: BLE001 - best effort while reporting an error
        return STATUS_NAMES.get(status, f"status {status}")


def load() -> ctypes.CDLL:
    """Load ``libiqa_hip.so`` and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is not built; run `python -m paper_2501_10653_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    f = ctypes.c_float
    cfgp = ctypes.POINTER(LaunchCfg)
    sigs = {
        "iqa_tiles": ([vp, vp, i64, i64, f, f, f, f, vp, vp, vp, vp], ctypes.c_int),
        "lisi_tiles": ([vp, vp, i64, i64, f, f, f, vp, vp], ctypes.c_int),
        "auglisi_tiles": ([vp, vp, i64, i64, f, vp, vp], ctypes.c_int),
        "iqa_default_cfg": ([i64, i64, vp, vp, cfgp], ctypes.c_int),
        "iqa_check_cfg": ([i64, i64, cfgp], ctypes.c_int),
        "iqa_tiles_cfg": ([vp, vp, i64, i64, f, f, f, f, vp, vp, vp, cfgp, vp], ctypes.c_int),
        "iqa_prepare": ([i64, i64, cfgp, vp], ctypes.c_int),
        "iqa_tiles_noalloc": ([vp, vp, i64, i64, f, f, f, f, vp, vp, vp, cfgp, vp],
                              ctypes.c_int),
        "iqa_launch_workgroups": ([i64, i64, cfgp], i64),
        "iqa_tiles_timeline": ([vp, vp, i64, i64, f, f, f, f, vp, vp, vp, cfgp, vp, i64, vp],
                               ctypes.c_int),
        "iqa_probe_empty": ([i64, ctypes.c_int32, vp], ctypes.c_int),
        "iqa_probe_read": ([vp, i64, vp, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp],
                           ctypes.c_int),
        "iqa_probe_read_timeline": ([vp, i64, vp, i64, ctypes.c_int32, ctypes.c_int32, vp, i64,
                                     vp], ctypes.c_int),
        "iqa_probe_last_hip_error": ([], ctypes.c_int),
        "iqa_wall_clock_khz": ([], i64),
        "iqa_read_ceiling": ([vp, i64, vp, i64, vp], ctypes.c_int),
        "iqa_merge_tiles": ([vp, i64, i64, f, f, f, vp, vp, vp, vp], ctypes.c_int),
        "iqa_tune_set": ([i64, i64, ctypes.c_int, cfgp], ctypes.c_int),
        "iqa_tune_clear": ([], None),
        "iqa_batch_default_waves": ([], ctypes.c_int64),
        "iqa_batch_cfg": ([i64, i64, cfgp], ctypes.c_int),
        "iqa_serve_cfg": ([i64, i64, cfgp], ctypes.c_int),
        "iqa_batch_describe": ([ctypes.POINTER(IqaPair), i64, vp, ctypes.POINTER(i64)],
                               ctypes.c_int),
        "iqa_tiles_batched": ([vp, i64, i64, i64, vp], ctypes.c_int),
        "iqa_tiles_batched_inline": ([vp, i64, i64, i64, vp], ctypes.c_int),
        "iqa_server_create": ([ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)], ctypes.c_int),
        "iqa_server_create_dry": ([ctypes.POINTER(ServerOpts), i64, ctypes.c_double,
                                   ctypes.POINTER(vp)], ctypes.c_int),
        "iqa_server_add_reference": ([vp, vp, i64, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "iqa_server_submit": ([vp, ctypes.POINTER(Request), i64], ctypes.c_int),
        "iqa_server_poll": ([vp, ctypes.POINTER(Completion), i64], ctypes.c_int64),
        "iqa_server_drain": ([vp, i64], ctypes.c_int),
        "iqa_server_get_stats": ([vp, ctypes.POINTER(ServerStats)], ctypes.c_int),
        "iqa_server_replay": ([vp, ctypes.POINTER(Request), ctypes.POINTER(i64), i64,
                               ctypes.POINTER(Completion), i64], ctypes.c_int),
        "iqa_server_destroy": ([vp], ctypes.c_int),
        "iqa_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "iqa_last_hip_error": ([], ctypes.c_int),
        "iqa_version": ([], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != IQA_OK:
        hip = load().iqa_last_hip_error() if status == 5 else 0
        raise IqaError(status, where, hip)
