"""Thin Python binding of libqms.so (argument marshalling only).

Every function here forwards to the C entry point of the same name in
``include/qms.h``; all sorting work runs in the HIP kernels of the library.
Tensors are torch tensors on a ROCm device (torch is used only for device
memory and streams).  If the library has not been built this module raises
on first use -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
# QMS_LIBRARY may point at another build of the same library (tuning runs)
LIB_PATH = os.environ.get("QMS_LIBRARY") or os.path.join(PKG, "libqms.so")

QMS_U32 = 0
QMS_F32 = 1
QMS_U64 = 2
QMS_F64 = 3
QMS_U32_LOG = 4  # uint32 keys compared by log(key) (an expensive comparison)

QMS_OK = 0
QMS_PENDING = 1
QMS_ERR_INVALID = -1
QMS_ERR_ALIGN = -2
QMS_ERR_NOMEM = -3
QMS_ERR_HIP = -4
QMS_ERR_BUDGET = -5
QMS_ERR_UNSUPPORTED = -6

# every extern "C" symbol declared in include/qms.h
EXPORTS = (
    "qms_sort", "qms_sort_pairs", "qms_sort_batch",
    "qms_server_create", "qms_server_submit", "qms_server_poll",
    "qms_server_get_stats", "qms_server_destroy",
    "qms_last_error", "qms_release_workspaces", "qms_last_schedule",
    "qms_get_tiles", "qms_profile_begin", "qms_profile_end", "qms_mom_pivot",
    "qms_set_tuning", "qms_get_tuning", "qms_sort_noalloc", "qms_batch_check",
)

QMS_SCHEDULE_WORDS = 6


class QmsError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("device", ctypes.c_int),
                ("max_batch", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("completed_keys", ctypes.c_uint64),
                ("peak_admitted_bytes", ctypes.c_uint64),
                ("waited_for_budget", ctypes.c_uint64), ("batches", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("merge_ways", ctypes.c_uint32), ("partition_tile", ctypes.c_uint32),
                ("chunk_span", ctypes.c_uint32), ("base_tile", ctypes.c_uint32),
                ("final_tile", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqms.so and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: the HIP library has not been built "
            "(run `python -m paper_1804_10062_amd.build`)")
    lib = ctypes.CDLL(path)
    vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.qms_sort.argtypes = [vp, u64, i32, vp]
    lib.qms_sort.restype = i32
    lib.qms_sort_noalloc.argtypes = [vp, u64, i32, vp]
    lib.qms_sort_noalloc.restype = i32
    lib.qms_sort_pairs.argtypes = [vp, vp, u64, i32, vp]
    lib.qms_sort_pairs.restype = i32
    lib.qms_sort_batch.argtypes = [vp, vp, vp, vp, u32, i32, vp]
    lib.qms_sort_batch.restype = i32
    lib.qms_batch_check.argtypes = [vp]
    lib.qms_batch_check.restype = i32
    lib.qms_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.qms_server_create.restype = i32
    lib.qms_server_submit.argtypes = [vp, vp, u64, i32, vp, u64p]
    lib.qms_server_submit.restype = i32
    lib.qms_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double)]
    lib.qms_server_poll.restype = i32
    lib.qms_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.qms_server_get_stats.restype = i32
    lib.qms_server_destroy.argtypes = [vp]
    lib.qms_server_destroy.restype = i32
    lib.qms_last_error.argtypes = []
    lib.qms_last_error.restype = ctypes.c_char_p
    lib.qms_release_workspaces.argtypes = []
    lib.qms_release_workspaces.restype = i32
    lib.qms_last_schedule.argtypes = [u64p, u64]
    lib.qms_last_schedule.restype = u64
    lib.qms_get_tiles.argtypes = [u32p, u32p, u32p]
    lib.qms_get_tiles.restype = None
    lib.qms_profile_begin.argtypes = []
    lib.qms_profile_begin.restype = i32
    lib.qms_profile_end.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    lib.qms_profile_end.restype = i32
    lib.qms_mom_pivot.argtypes = [vp, u64, i32, vp, vp]
    lib.qms_mom_pivot.restype = i32
    lib.qms_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.qms_set_tuning.restype = i32
    lib.qms_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.qms_get_tuning.restype = i32
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().qms_last_error().decode()


def _check(code: int, where: str) -> int:
    if code < 0:
        raise QmsError(code, where, last_error())
    return code


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return QMS_F32
    if t.dtype in (torch.int32, torch.uint32):
        return QMS_U32
    if t.dtype == torch.float64:
        return QMS_F64
    if t.dtype in (torch.int64, torch.uint64):
        return QMS_U64
    raise TypeError("keys must be float32/float64 or 32/64-bit integers (bit patterns of "
                    f"unsigned keys), got {t.dtype}")


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def qms_sort(keys, stream=None, dtype: Optional[int] = None) -> None:
    """Sort a 1-D device tensor of 32- or 64-bit keys in place.

    uint32/int32 (uint64/int64) tensors are sorted as unsigned integers of
    their width (a signed tensor is taken as the bit pattern of unsigned
    keys); float32 and float64 tensors by the IEEE-754 total order."""
    _check_tensor(keys, "keys")
    lib = load_library()
    dt = _dtype_code(keys) if dtype is None else dtype
    _check(lib.qms_sort(keys.data_ptr(), keys.numel(), dt, _stream_handle(stream)), "qms_sort")


def qms_sort_noalloc(keys, stream=None, dtype: Optional[int] = None) -> None:
    """qms_sort without any allocation (at most 2^28 keys; the library's
    fixed device scratch array instead of a cached workspace)."""
    _check_tensor(keys, "keys")
    lib = load_library()
    dt = _dtype_code(keys) if dtype is None else dtype
    _check(lib.qms_sort_noalloc(keys.data_ptr(), keys.numel(), dt, _stream_handle(stream)),
           "qms_sort_noalloc")


def qms_sort_pairs(keys, vals, stream=None, dtype: Optional[int] = None) -> None:
    """Sort keys in place, permuting the uint32 payload tensor ``vals`` with them."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals.numel() != keys.numel() or vals.element_size() != 4:
        raise ValueError("vals must hold one 32-bit word per key")
    lib = load_library()
    dt = _dtype_code(keys) if dtype is None else dtype
    _check(lib.qms_sort_pairs(keys.data_ptr(), vals.data_ptr(), keys.numel(), dt,
                              _stream_handle(stream)), "qms_sort_pairs")


def qms_sort_batch(keys, offsets, vals=None, host_offsets=None, stream=None,
                   dtype: Optional[int] = None) -> None:
    """Sort every segment [offsets[j], offsets[j+1]) of ``keys`` in place.

    ``offsets`` is a device uint64/int64 tensor of num_segments + 1 entries;
    ``host_offsets`` an optional numpy copy of it."""
    _check_tensor(keys, "keys")
    _check_tensor(offsets, "offsets")
    if vals is not None:
        _check_tensor(vals, "vals")
    lib = load_library()
    dt = _dtype_code(keys) if dtype is None else dtype
    hp = None
    if host_offsets is not None:
        import numpy as np
        host_offsets = np.ascontiguousarray(host_offsets, dtype=np.uint64)
        hp = host_offsets.ctypes.data
    nseg = offsets.numel() - 1
    _check(lib.qms_sort_batch(keys.data_ptr(), None if vals is None else vals.data_ptr(),
                              offsets.data_ptr(), hp, nseg, dt, _stream_handle(stream)),
           "qms_sort_batch")


def qms_batch_check(stream=None) -> None:
    """Wait for the stream and raise if a batch sorted on it left segments
    unsorted (a check of the library's device-side schedule)."""
    _check(load_library().qms_batch_check(_stream_handle(stream)), "qms_batch_check")


def qms_last_schedule(max_rounds: int = 4096):
    """Per-round log of the last single-array sort on this thread: a list of
    (s, n_less, n_equal, n_greater, merge_levels, pivot_rule) with
    pivot_rule 0 = median-of-3, 1 = median of the medians of three."""
    lib = load_library()
    w = QMS_SCHEDULE_WORDS
    buf = (ctypes.c_uint64 * (w * max_rounds))()
    n = lib.qms_last_schedule(buf, max_rounds)
    return [tuple(buf[w * i:w * i + w]) for i in range(min(n, max_rounds))]


def qms_mom_pivot(keys, stream=None, dtype: Optional[int] = None) -> int:
    """Median of the medians of the triples of `keys` (1-D device tensor of
    32- or 64-bit keys, dtype as in qms_sort), as the bit pattern of the
    pivot (32 or 64 bits by the key width)."""
    _check_tensor(keys, "keys")
    dt = _dtype_code(keys) if dtype is None else dtype
    out = ctypes.c_uint64() if dt in (QMS_U64, QMS_F64) else ctypes.c_uint32()
    _check(load_library().qms_mom_pivot(keys.data_ptr(), keys.numel(), dt,
                                        ctypes.byref(out), _stream_handle(stream)),
           "qms_mom_pivot")
    return out.value


def qms_set_tuning(merge_ways: int, partition_tile: int, chunk_span: int,
                   base_tile: Optional[int] = None, final_tile: Optional[int] = None) -> None:
    """Set the run-time tunables (qms.h); base_tile / final_tile left as
    None keep their current values."""
    if base_tile is None or final_tile is None:
        cur = qms_get_tuning()
        base_tile = cur["base_tile"] if base_tile is None else base_tile
        final_tile = cur["final_tile"] if final_tile is None else final_tile
    t = Tuning(merge_ways, partition_tile, chunk_span, base_tile, final_tile)
    _check(load_library().qms_set_tuning(ctypes.byref(t)), "qms_set_tuning")


def qms_get_tuning() -> dict:
    t = Tuning()
    _check(load_library().qms_get_tuning(ctypes.byref(t)), "qms_get_tuning")
    return t.as_dict()


def qms_get_tiles():
    lib = load_library()
    a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.qms_get_tiles(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return {"base_tile": a.value, "merge_tile": b.value, "partition_tile": c.value}


def qms_profile_begin() -> None:
    _check(load_library().qms_profile_begin(), "qms_profile_begin")


def qms_profile_end() -> dict:
    """{class: {"launches", "total_ms", "bytes"}} for the sorts since begin."""
    lib = load_library()
    buf = (KernelStat * 48)()
    n = ctypes.c_int()
    _check(lib.qms_profile_end(buf, 48, ctypes.byref(n)), "qms_profile_end")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "bytes": buf[i].bytes} for i in range(n.value)}


def qms_release_workspaces() -> None:
    _check(load_library().qms_release_workspaces(), "qms_release_workspaces")


class Server:
    """The request loop of the library (qms_server_* entry points)."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0, max_batch: int = 0):
        lib = load_library()
        cfg = ServerConfig(hbm_budget_bytes, device, max_batch)
        h = ctypes.c_void_p()
        _check(lib.qms_server_create(ctypes.byref(cfg), ctypes.byref(h)), "qms_server_create")
        self._h = h
        self._lib = lib

    def submit(self, keys, dtype: Optional[int] = None, stream=None) -> int:
        """Lend ``keys`` to the server; it sorts them after the work already
        enqueued on ``stream`` (default: the current stream) has run."""
        _check_tensor(keys, "keys")
        dt = _dtype_code(keys) if dtype is None else dtype
        t = ctypes.c_uint64()
        _check(self._lib.qms_server_submit(self._h, keys.data_ptr(), keys.numel(), dt,
                                           _stream_handle(stream), ctypes.byref(t)),
               "qms_server_submit")
        return t.value

    def poll(self, ticket: int):
        """Returns (status, latency_seconds_or_None)."""
        lat = ctypes.c_double(-1.0)
        rc = self._lib.qms_server_poll(self._h, ticket, ctypes.byref(lat))
        if rc < 0:
            raise QmsError(rc, "qms_server_poll", last_error())
        return rc, (lat.value if rc == QMS_OK else None)

    def stats(self) -> dict:
        s = ServerStats()
        _check(self._lib.qms_server_get_stats(self._h, ctypes.byref(s)), "qms_server_get_stats")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            _check(self._lib.qms_server_destroy(self._h), "qms_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
