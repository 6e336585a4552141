"""CPU oracle for QuickMergesort with median-of-3 pivots -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it
and shares no code with it (see ``qms_oracle.c`` for the algorithm, the
readings of the paper it takes, and the counters).

The C source is compiled with gcc into ``oracle/_build/liboracle.so``; this
module loads it with ctypes and offers numpy-level helpers:

* ``sort(keys, vals=None, counted=True)`` -- QuickMergesort (Fig. 2 of the
  paper, median-of-3, X_THRESH = 2) on copies of the inputs; returns the
  sorted arrays and the (comparisons, moves) counters.
* ``sort_segments`` -- the same, independently per segment.
* ``sort_x(keys, x_thresh=None)`` -- QuickMergeXsort: msort hands ranges
  shorter than ``x_thresh`` (default ceil(sqrt(n))) to X = CleverQuicksort
  (Sec. "QuickMergeXsort"); ``x_thresh = 2`` is QuickMergesort.
* ``clever_quicksort(keys)`` -- X alone, median-of-3 Quicksort.
* ``partition``, ``out``, ``msort``, ``merge`` -- the individual routines of
  Fig. 2, for pinning them one by one; ``msort_x`` is msort with X.
* ``mom_pivot(keys)`` -- the worst-case pivot of the paper's
  MoMQuickMergesort: the lower median of the medians of the triples.
* ``order_statistic_ok(x, k, v)`` -- whether ``v`` is the element of rank
  ``k`` of ``x`` by the plain counting definition (for checking sampled
  outputs at sizes where a full oracle sort is too slow).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qms_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle (counting and timing builds) into one shared object."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(_BUILD, exist_ok=True)
    objs = []
    for bits in (32, 64):
        for counting in (1, 0):
            obj = os.path.join(_BUILD, f"qms_oracle_{bits}_{counting}.o")
            subprocess.check_call([
                "gcc", "-std=c11", "-O2", "-fPIC", "-Wall", "-Wextra",
                f"-DQMSO_COUNTING={counting}", f"-DQMSO_KEY_BITS={bits}", "-c", _SRC,
                "-o", obj,
            ])
            objs.append(obj)
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-shared", "-o", tmp] + objs)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Counters(ctypes.Structure):
    _fields_ = [("comparisons", ctypes.c_uint64), ("moves", ctypes.c_uint64)]


class Counts(NamedTuple):
    comparisons: int
    moves: int


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    cp = ctypes.POINTER(_Counters)
    sz = ctypes.c_size_t
    for name in ("qmso_sort", "qmso_fast_sort"):
        f = getattr(lib, name)
        f.argtypes = [u32p, u32p, sz, ctypes.c_int, cp]
        f.restype = None
    # 64-bit keys: the same routines compiled for uint64 keys
    for name in ("qmso64_sort", "qmso64_fast_sort", "qmso64_clever_quicksort",
                 "qmso64_fast_clever_quicksort"):
        f = getattr(lib, name)
        f.argtypes = [u64p, u32p, sz, ctypes.c_int, cp]
        f.restype = None
    for name in ("qmso64_sort_x", "qmso64_fast_sort_x"):
        f = getattr(lib, name)
        f.argtypes = [u64p, u32p, sz, ctypes.c_int, sz, cp]
        f.restype = None
    for name in ("qmso64_sort_segments", "qmso64_fast_sort_segments"):
        f = getattr(lib, name)
        f.argtypes = [u64p, u32p, u64p, sz, ctypes.c_int, cp]
        f.restype = None
    for name in ("qmso_sort_x", "qmso_fast_sort_x"):
        f = getattr(lib, name)
        f.argtypes = [u32p, u32p, sz, ctypes.c_int, sz, cp]
        f.restype = None
    for name in ("qmso_clever_quicksort", "qmso_fast_clever_quicksort"):
        f = getattr(lib, name)
        f.argtypes = [u32p, u32p, sz, ctypes.c_int, cp]
        f.restype = None
    for name in ("qmso_sort_segments", "qmso_fast_sort_segments"):
        f = getattr(lib, name)
        f.argtypes = [u32p, u32p, u64p, sz, ctypes.c_int, cp]
        f.restype = None
    lib.qmso_partition.argtypes = [u32p, u32p, sz, sz, cp]
    lib.qmso_partition.restype = sz
    lib.qmso_out.argtypes = [u32p, u32p, sz, sz, sz, cp]
    lib.qmso_out.restype = None
    lib.qmso_msort.argtypes = [u32p, u32p, sz, sz, sz, cp]
    lib.qmso_msort.restype = None
    lib.qmso_msort_x.argtypes = [u32p, u32p, sz, sz, sz, sz, cp]
    lib.qmso_msort_x.restype = None
    lib.qmso_merge.argtypes = [u32p, u32p, sz, sz, sz, sz, cp]
    lib.qmso_merge.restype = None
    lib.qmso_mom_pivot.argtypes = [u32p, sz, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.qmso_mom_pivot.restype = ctypes.c_uint32
    lib.qmso64_mom_pivot.argtypes = [u64p, sz, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.qmso64_mom_pivot.restype = ctypes.c_uint64
    _lib = lib
    return lib


def _as_words(a: np.ndarray) -> tuple[np.ndarray, int]:
    """Return a contiguous unsigned copy of the key words (32 or 64 bits) and
    the float flag."""
    a = np.asarray(a)
    if a.dtype == np.float32:
        return np.ascontiguousarray(a).view(np.uint32).copy(), 1
    if a.dtype == np.uint32:
        return np.ascontiguousarray(a).copy(), 0
    if a.dtype == np.float64:
        return np.ascontiguousarray(a).view(np.uint64).copy(), 1
    if a.dtype == np.uint64:
        return np.ascontiguousarray(a).copy(), 0
    raise TypeError(f"oracle sorts uint32/uint64 or float32/float64 keys, got {a.dtype}")


def _ptr(a):
    if a is None:
        return None
    if a.dtype == np.uint64:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _wide(words: np.ndarray) -> bool:
    return words.dtype == np.uint64


def _floats(words: np.ndarray, is_f: int) -> np.ndarray:
    if not is_f:
        return words
    return words.view(np.float64 if _wide(words) else np.float32)


def sort(keys, vals=None, counted: bool = True):
    """QuickMergesort copies of ``keys`` (and ``vals``); returns (keys, vals, Counts)."""
    lib = _load()
    words, is_f32 = _as_words(keys)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if v is not None and v.shape != words.shape:
        raise ValueError("keys and vals differ in length")
    c = _Counters()
    pre = "qmso64_" if _wide(words) else "qmso_"
    fn = getattr(lib, pre + ("sort" if counted else "fast_sort"))
    fn(_ptr(words), _ptr(v), words.size, is_f32, ctypes.byref(c))
    return _floats(words, is_f32), v, Counts(int(c.comparisons), int(c.moves))


def sqrt_threshold(n: int) -> int:
    """ceil(sqrt(n)): the X_THRESH of QuickMergeXsort's sqrt(n) configuration."""
    r = int(np.floor(np.sqrt(float(n))))
    while r * r < n:
        r += 1
    while r > 0 and (r - 1) * (r - 1) >= n:
        r -= 1
    return max(r, 2)


def sort_x(keys, vals=None, x_thresh: int | None = None, counted: bool = True):
    """QuickMergeXsort copies of the inputs with X = CleverQuicksort called on
    msort ranges shorter than ``x_thresh`` (default ceil(sqrt(n))); returns
    (keys, vals, Counts)."""
    lib = _load()
    words, is_f32 = _as_words(keys)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if v is not None and v.shape != words.shape:
        raise ValueError("keys and vals differ in length")
    xt = sqrt_threshold(words.size) if x_thresh is None else int(x_thresh)
    if xt < 2:
        raise ValueError("x_thresh must be at least 2")
    c = _Counters()
    pre = "qmso64_" if _wide(words) else "qmso_"
    fn = getattr(lib, pre + ("sort_x" if counted else "fast_sort_x"))
    fn(_ptr(words), _ptr(v), words.size, is_f32, xt, ctypes.byref(c))
    return _floats(words, is_f32), v, Counts(int(c.comparisons), int(c.moves))


def clever_quicksort(keys, vals=None, counted: bool = True):
    """X alone: median-of-3 Quicksort of copies; returns (keys, vals, Counts)."""
    lib = _load()
    words, is_f32 = _as_words(keys)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    c = _Counters()
    pre = "qmso64_" if _wide(words) else "qmso_"
    fn = getattr(lib, pre + ("clever_quicksort" if counted else "fast_clever_quicksort"))
    fn(_ptr(words), _ptr(v), words.size, is_f32, ctypes.byref(c))
    return _floats(words, is_f32), v, Counts(int(c.comparisons), int(c.moves))


def sort_segments(keys, offsets, vals=None, counted: bool = False):
    """Sort every segment [offsets[j], offsets[j+1]) of copies of the inputs."""
    lib = _load()
    words, is_f32 = _as_words(keys)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    c = _Counters()
    pre = "qmso64_" if _wide(words) else "qmso_"
    fn = getattr(lib, pre + ("sort_segments" if counted else "fast_sort_segments"))
    fn(_ptr(words), _ptr(v), off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
       off.size - 1, is_f32, ctypes.byref(c))
    return _floats(words, is_f32), v, Counts(int(c.comparisons), int(c.moves))


def sort_inplace_fast(words: np.ndarray, is_f32: bool) -> None:
    """Timing build, sorting a caller-owned contiguous uint32 array in place."""
    lib = _load()
    assert words.dtype == np.uint32 and words.flags.c_contiguous
    lib.qmso_fast_sort(_ptr(words), None, words.size, int(is_f32), None)


def partition(keys, lo: int, hi: int, vals=None):
    """Median-of-3 partition of [lo, hi) of a copy; returns (keys, vals, b, Counts)."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if not (0 <= lo and hi <= k.size and hi - lo >= 3):
        raise ValueError("partition needs 3 <= hi - lo within the array")
    c = _Counters()
    b = lib.qmso_partition(_ptr(k), _ptr(v), lo, hi, ctypes.byref(c))
    return k, v, int(b), Counts(int(c.comparisons), int(c.moves))


def out(keys, begin: int, end: int, temp: int, vals=None):
    """Fig. 2 ``out`` on a copy: sort [begin, end) using ceil(n/2) cells at temp."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    n = end - begin
    r = n - n // 2
    if n > 1 and not (0 <= begin <= end <= k.size and 0 <= temp
                      and temp + r <= k.size
                      and (temp + r <= begin or temp >= end)):
        raise ValueError("out: buffer must hold ceil(n/2) cells outside [begin, end)")
    c = _Counters()
    lib.qmso_out(_ptr(k), _ptr(v), begin, end, temp, ctypes.byref(c))
    return k, v, Counts(int(c.comparisons), int(c.moves))


def msort(keys, begin: int, end: int, target: int, vals=None):
    """Fig. 2 ``msort`` on a copy: sort [begin, end) into [target, target+n)."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    n = end - begin
    if not (0 <= begin <= end <= k.size and 0 <= target and target + n <= k.size):
        raise ValueError("msort: ranges out of the array")
    c = _Counters()
    lib.qmso_msort(_ptr(k), _ptr(v), begin, end, target, ctypes.byref(c))
    return k, v, Counts(int(c.comparisons), int(c.moves))


def msort_x(keys, begin: int, end: int, target: int, x_thresh: int, vals=None):
    """QuickMergeXsort's msort on a copy: X below ``x_thresh``."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    n = end - begin
    if not (0 <= begin <= end <= k.size and 0 <= target and target + n <= k.size):
        raise ValueError("msort: ranges out of the array")
    c = _Counters()
    lib.qmso_msort_x(_ptr(k), _ptr(v), begin, end, target, max(2, int(x_thresh)),
                     ctypes.byref(c))
    return k, v, Counts(int(c.comparisons), int(c.moves))


def merge(keys, begin1: int, end1: int, target: int, endtarget: int, vals=None):
    """Fig. 2 ``merge`` on a copy (run2 already at target + len1)."""
    lib = _load()
    k = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if not (end1 > begin1 and endtarget <= k.size):
        raise ValueError("merge: run1 must be non-empty and the target in range")
    c = _Counters()
    lib.qmso_merge(_ptr(k), _ptr(v), begin1, end1, target, endtarget,
                   ctypes.byref(c))
    return k, v, Counts(int(c.comparisons), int(c.moves))


def mom_pivot(keys: np.ndarray) -> int:
    """Median of the floor(n/3) medians of (keys[3i], keys[3i+1], keys[3i+2])
    (Sec. "Worst-Case Efficient QuickMergeSort", reading R7), as the bit
    pattern of the pivot (32 or 64 bits by the key width); float keys are
    compared by the total order.  Other integer arrays are taken as uint32."""
    x = np.ascontiguousarray(keys)
    if x.size < 3:
        raise ValueError("the pivot needs n >= 3")
    if x.dtype not in (np.float32, np.uint32, np.float64, np.uint64):
        x = x.astype(np.uint32, copy=False)
    words, is_f = _as_words(x)
    lib = _load()
    ok = ctypes.c_int()
    fn = lib.qmso64_mom_pivot if _wide(words) else lib.qmso_mom_pivot
    p = fn(_ptr(words), words.size, is_f, ctypes.byref(ok))
    if not ok.value:
        raise MemoryError("oracle mom_pivot")
    return int(p)


def order_statistic_ok(x: np.ndarray, k: int, value) -> bool:
    """True iff ``value`` is the rank-``k`` element (0-based) of ``x``.

    Plain definition: #{x < v} <= k < #{x <= v}, with the comparison taken
    in the key order the sort uses (unsigned for uint32; for float32 the
    IEEE-754 total order, evaluated on the bit patterns).
    """
    x = np.asarray(x)
    if x.dtype == np.float32:
        xb = x.view(np.uint32).astype(np.int64)
        vb = int(np.asarray(value, dtype=np.float32).view(np.uint32))
        # total order as a signed comparison of sign-magnitude integers
        xs = np.where(xb >= 2**31, -(xb - 2**31) - 1, xb)
        vs = -(vb - 2**31) - 1 if vb >= 2**31 else vb
        lt = int(np.count_nonzero(xs < vs))
        le = int(np.count_nonzero(xs <= vs))
    else:
        v = np.uint32(value)
        lt = int(np.count_nonzero(x < v))
        le = int(np.count_nonzero(x <= v))
    return lt <= k < le
