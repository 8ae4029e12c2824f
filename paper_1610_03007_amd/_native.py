"""ctypes binding of ``libsa_mi355x.so`` (the C ABI declared in include/sa.h).

Argument marshalling only: every step of the suffix-array build runs in the HIP
library. PyTorch supplies device memory (CUDA tensors on ROCm) and the current
stream. There is no CPU fallback: if the library is missing or cannot be
loaded, importing it raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

from . import build_ext

SA_OK, SA_EINVAL, SA_ENOMEM, SA_ETOOBIG, SA_EDEVICE, SA_EBUSY = range(6)
SA_MAX_ROUNDS = 64
SA_NOALLOC_MAX_N = 1 << 20
KERNEL_KINDS = {
    "sort_pass": 0,
    "histogram": 1,
    "rerank": 2,
    "pack_text": 3,
    "pack_pairs": 4,
    "other": 5,
    "isa_scatter": 6,
}
ISA_MODES = {"auto": 0, "eager": 1, "lazy": 2}

EXPORTED = [
    "sa_ctx_create", "sa_ctx_destroy", "sa_build", "sa_build_noalloc", "sa_build_batch",
    "sa_last_build_info",
    "sa_build_rounds", "sa_build_sorted_pairs", "sa_build_dc3", "sa_build_dc7",
    "sa_radix_sort_pairs", "sa_workspace_bytes", "sa_ctx_set_trace", "sa_ctx_reset_stats",
    "sa_ctx_set_isa_mode", "sa_ctx_set_tuning", "sa_ctx_get_tuning", "sa_ctx_tuning_source",
    "sa_tune", "sa_tune_save", "sa_tune_lookup",
    "sa_server_create", "sa_server_destroy", "sa_server_submit", "sa_server_poll",
    "sa_server_stats",
    "sa_ctx_get_kernel_stats", "sa_strerror",
    "sa_lcp", "sa_bwt", "sa_fm_create", "sa_fm_count", "sa_fm_info", "sa_fm_destroy",
]


class BuildInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("rounds", ctypes.c_uint32),
        ("sigma", ctypes.c_uint32),
        ("code_bits", ctypes.c_uint32),
        ("chars0", ctypes.c_uint32),
        ("prefix_len", ctypes.c_uint64),
        ("lazy_isa", ctypes.c_uint32),
        ("graph_rounds", ctypes.c_uint32),
        ("dense_rounds", ctypes.c_uint64),
        ("active", ctypes.c_uint64 * SA_MAX_ROUNDS),
        ("passes_run", ctypes.c_uint32 * SA_MAX_ROUNDS),
        ("key_bits", ctypes.c_uint32 * SA_MAX_ROUNDS),
    ]

    def as_dict(self) -> dict:
        r = int(self.rounds)
        return {
            "n": int(self.n), "rounds": r, "sigma": int(self.sigma),
            "code_bits": int(self.code_bits), "chars0": int(self.chars0),
            "prefix_len": int(self.prefix_len),
            "lazy_isa": bool(self.lazy_isa),
            "graph_rounds": int(self.graph_rounds),
            "dense_rounds": [k for k in range(r) if (int(self.dense_rounds) >> k) & 1],
            "active": [int(x) for x in self.active[:r]],
            "passes_run": [int(x) for x in self.passes_run[:r]],
            "key_bits": [int(x) for x in self.key_bits[:r]],
        }


class Tuning(ctypes.Structure):
    _fields_ = [("sort_items", ctypes.c_uint32), ("lazy_ratio", ctypes.c_uint32),
                ("round0_full", ctypes.c_uint32), ("sort_wgs_per_cu", ctypes.c_uint32),
                ("sort_block", ctypes.c_uint32), ("sort_match", ctypes.c_uint32),
                ("radix_bits", ctypes.c_uint32), ("rounds_ahead", ctypes.c_uint32),
                ("round_graphs", ctypes.c_uint32), ("prefix_mult", ctypes.c_uint32),
                ("isa_direct", ctypes.c_uint32)]


TUNING_KNOBS = ("sort_items", "lazy_ratio", "round0_full", "sort_wgs_per_cu", "sort_block",
                "sort_match", "radix_bits", "rounds_ahead", "round_graphs", "prefix_mult",
                "isa_direct")


def tuning_dict(t: "Tuning") -> dict:
    return {k: int(getattr(t, k)) for k in TUNING_KNOBS}


def tune_lookup(path: str, arch: str, mode: str, n: int, code_bits: int = 0):
    """(found, tuning dict) a build would take from the cache file at ``path``."""
    t = Tuning()
    found = ctypes.c_int(0)
    check(lib().sa_tune_lookup(path.encode(), arch.encode(), mode.encode(), n, code_bits,
                               ctypes.byref(t), ctypes.byref(found)), "sa_tune_lookup")
    return bool(found.value), tuning_dict(t)


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("suffixes", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("busy_ms", ctypes.c_double), ("queued", ctypes.c_uint64),
                ("running", ctypes.c_uint64), ("slots", ctypes.c_uint64),
                ("arena_positions", ctypes.c_uint64)]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class SAError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} (status {status})")


_lock = threading.Lock()
_lib = None


def _declare(lib: ctypes.CDLL) -> None:
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "sa_ctx_create": ([ctypes.POINTER(vp), i32, ctypes.c_char_p], i32),
        "sa_ctx_destroy": ([vp], i32),
        "sa_build": ([vp, vp, u64, u32, vp, vp], i32),
        "sa_build_noalloc": ([vp, vp, u64, u32, vp, vp], i32),
        "sa_build_batch": ([vp, vp, vp, u32, vp, vp], i32),
        "sa_last_build_info": ([vp, ctypes.POINTER(BuildInfo)], i32),
        "sa_build_rounds": ([vp, vp, u64, u32, vp, vp, vp], i32),
        "sa_build_sorted_pairs": ([vp, vp, u64, u32, vp, vp, u32, vp], i32),
        "sa_build_dc3": ([vp, vp, u64, vp, vp, vp], i32),
        "sa_build_dc7": ([vp, vp, u64, vp, vp, vp], i32),
        "sa_radix_sort_pairs": ([vp, vp, vp, u64, u32, vp], i32),
        "sa_workspace_bytes": ([u64, u32], ctypes.c_size_t),
        "sa_ctx_set_trace": ([vp, i32], i32),
        "sa_ctx_set_isa_mode": ([vp, i32], i32),
        "sa_ctx_set_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "sa_ctx_get_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "sa_ctx_tuning_source": ([vp, ctypes.POINTER(i32)], i32),
        "sa_tune": ([vp, vp, vp, u32, vp, vp, u32, ctypes.POINTER(Tuning),
                     ctypes.POINTER(ctypes.c_double)], i32),
        "sa_tune_save": ([vp, ctypes.c_char_p], i32),
        "sa_tune_lookup": ([ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, u64, u32,
                            ctypes.POINTER(Tuning), ctypes.POINTER(i32)], i32),
        "sa_ctx_reset_stats": ([vp], i32),
        "sa_ctx_get_kernel_stats": ([vp, i32, ctypes.POINTER(KernelStats)], i32),
        "sa_strerror": ([i32], ctypes.c_char_p),
        "sa_server_create": ([ctypes.POINTER(vp), i32, u64, u64], i32),
        "sa_server_destroy": ([vp], i32),
        "sa_server_submit": ([vp, vp, u64, ctypes.POINTER(u64)], i32),
        "sa_server_poll": ([vp, u64, vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)],
                           i32),
        "sa_server_stats": ([vp, ctypes.POINTER(ServerStats)], i32),
        "sa_lcp": ([vp, vp, u64, vp, vp, vp], i32),
        "sa_bwt": ([vp, vp, u64, vp, vp, ctypes.POINTER(u64), vp], i32),
        "sa_fm_create": ([ctypes.POINTER(vp), vp, vp, u64, vp, vp], i32),
        "sa_fm_count": ([vp, vp, vp, u32, vp, vp], i32),
        "sa_fm_info": ([vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32),
                        ctypes.POINTER(u64)], i32),
        "sa_fm_destroy": ([vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


def lib() -> ctypes.CDLL:
    """Load the HIP library, building it first only if no build exists."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(build_ext.LIB):
                build_ext.build()
            handle = ctypes.CDLL(build_ext.LIB)
            _declare(handle)
            _lib = handle
        return _lib


def _strerror(status: int) -> str:
    try:
        return lib().sa_strerror(status).decode()
    except Exception:  # pragma: no cover - only when the library itself is broken
        return "unknown"


def check(status: int, what: str) -> None:
    if status != SA_OK:
        raise SAError(status, what)
