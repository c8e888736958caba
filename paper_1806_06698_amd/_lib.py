"""ctypes binding of libsyev3.so (the C ABI in include/syev3.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsyev3.so")

F64 = 0
F32_REFINE = 1
F32 = 2
SOA = 0
AOS = 1
AOS9 = 2
FLAG_SIMPLIFIED_DEFLATION = 1
FLAG_NO_H_GUARD = 2
FLAG_NEWTON = 4
FLAG_PAPER_BG = 8
FLAG_REFINE_CONVERGE = 16
FLAG_NO_SCALE = 32

E = {
    0: "OK", -1: "E_N", -2: "E_NULL", -3: "E_DTYPE", -4: "E_LAYOUT",
    -5: "E_ALIAS", -6: "E_HIP", -7: "E_FLAGS", -8: "E_BUDGET", -9: "E_AGAIN",
    -10: "E_STATE", -11: "E_TIMEOUT", -12: "E_NOMEM", -13: "E_SEGMENTS",
}
SEGMENTS_MAX = 1024
E_AGAIN = -9


class Syev3Error(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = f"{where}: {E.get(code, code)} ({strerror(code)})" if where else strerror(code)
        super().__init__(msg)


_lib = None


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64),
                ("max_requests", ctypes.c_int32),
                ("max_inflight_ticks", ctypes.c_int32),
                ("max_segments_per_tick", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


class RequestBuffers(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("lam", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("dtype", ctypes.c_int32)]


class Segment(ctypes.Structure):
    """syev3_segment: one request of syev3_solve_segments_noalloc."""
    _fields_ = [("n", ctypes.c_int64), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("lam", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("matrices_completed", ctypes.c_int64),
                ("pool_bytes_in_use", ctypes.c_uint64),
                ("pool_bytes_peak", ctypes.c_uint64),
                ("acquire_rejections", ctypes.c_int64),
                ("inflight_ticks_peak", ctypes.c_int32),
                ("segments_per_tick_peak", ctypes.c_int32),
                ("busy_seconds", ctypes.c_double),
                ("queue_depth", ctypes.c_int64),
                ("queue_depth_peak", ctypes.c_int64),
                ("failed", ctypes.c_int64)]


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1806_06698_amd.build` "
            "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
    L.batched_syev3.argtypes = [i64, vp, vp, vp, i32, vp]
    L.batched_syev3.restype = i32
    L.batched_syev3_ex.argtypes = [i64, vp, i64, i32, vp, vp, i32, u32, vp]
    L.batched_syev3_ex.restype = i32
    L.batched_syev3_inplace.argtypes = [i64, vp, vp, i32, vp]
    L.batched_syev3_inplace.restype = i32
    L.batched_syev3_info.argtypes = [i64, vp, i64, i32, vp, vp, i32, u32, vp, vp]
    L.batched_syev3_info.restype = i32
    L.batched_syev3_strided.argtypes = [i64, vp, i64, vp, i64, vp, i64, i32, u32, vp]
    L.batched_syev3_strided.restype = i32
    L.syev3_stream_reference.argtypes = [i64, vp, vp, vp, i32, vp]
    L.syev3_stream_reference.restype = i32
    L.syev3_stream_probe.argtypes = [i64, vp, vp, vp, i32, u32, vp]
    L.syev3_stream_probe.restype = i32
    L.syev3_solve_segments_noalloc.argtypes = [i32, ctypes.POINTER(Segment), vp]
    L.syev3_solve_segments_noalloc.restype = i32
    L.syev3_strerror.argtypes = [i32]
    L.syev3_strerror.restype = ctypes.c_char_p
    L.syev3_version.argtypes = []
    L.syev3_version.restype = i32
    if hasattr(L, "syev3_server_create"):
        L.syev3_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
        L.syev3_server_default_opts.restype = None
        L.syev3_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.syev3_server_create.restype = i32
        L.syev3_server_destroy.argtypes = [vp]
        L.syev3_server_destroy.restype = i32
        L.syev3_server_acquire.argtypes = [vp, i64, i32, i32, ctypes.POINTER(RequestBuffers)]
        L.syev3_server_acquire.restype = i64
        L.syev3_server_submit.argtypes = [vp, i64, vp]
        L.syev3_server_submit.restype = i32
        L.syev3_server_poll.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
        L.syev3_server_poll.restype = i32
        L.syev3_server_wait.argtypes = [vp, i64, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double)]
        L.syev3_server_wait.restype = i32
        L.syev3_server_release.argtypes = [vp, i64]
        L.syev3_server_release.restype = i32
        L.syev3_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.syev3_server_get_stats.restype = i32
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().syev3_strerror(code).decode()
    except RuntimeError:
        return E.get(code, str(code))


def check(rc: int, where: str) -> int:
    if rc < 0:
        raise Syev3Error(rc, where)
    return rc
