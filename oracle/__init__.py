"""CPU oracle for suffix-array construction by prefix doubling.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path (the HIP library and
its binding) never does, and shares no code with it.

The arithmetic lives in ``oracle.cpp`` (plain C++17, ``std::sort``). This module
compiles it with g++ on demand and wraps it with ctypes over numpy arrays:

* :func:`sa` -- plain prefix doubling (paper Alg. 1 with the inverse-suffix-array
  pairing of Alg. 4), no discarding; 1-based names with 0 as the sentinel.
* :func:`pd_names` -- the names after a given number of doubling sorts.
* :func:`pa_names`, :func:`pa_sa` -- prefix a-tupling (a = 4: the paper's prefix
  quadrupling): names of single characters, then sorts of a-tuples of names.
* :func:`opk_order`, :func:`pdd_sa`, :func:`pdd_round` -- prefix doubling with
  discarding by sorting (Alg. 5 with the comparator of Eq. 1 and Alg. 6): the
  comparator's position order, the suffix array with per-round item counts, and
  the working items of one round.
* :func:`dc3_sample_ranks`, :func:`dcx_sample_ranks` -- the ranks among
  themselves of the suffixes that start in a difference cover sample (DC3:
  positions not divisible by 3; DC7: positions 0, 1, 3 mod 7), by definition.
* :func:`prefix_ranks` -- the closed form of the names for prefix length ``h``:
  1 + the number of suffixes whose padded length-``h`` prefix is smaller.
* :func:`brute_sa` -- the definition: sort all suffixes lexicographically.
* :func:`check_sa` -- linear-time suffix-array check (permutation plus an
  adjacent-pair test against the inverse of the array under test).
* :func:`lcp`, :func:`bwt`, :func:`sa_interval` -- index structures from a
  suffix array, each by its definition: adjacent-suffix common prefixes, the
  Burrows-Wheeler column of text$, and the suffix-array range of a pattern.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
LIB_SEQ = os.path.join(_HERE, "liboracle.so")
LIB_PAR = os.path.join(_HERE, "liboracle_par.so")

_lock = threading.Lock()
_libs: dict[bool, ctypes.CDLL] = {}


def build(parallel: bool | None = None) -> None:
    """Compile the sequential and the OpenMP (GNU parallel sort) builds."""
    targets = [False, True] if parallel is None else [parallel]
    for par in targets:
        out = LIB_PAR if par else LIB_SEQ
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out + ".tmp", _SRC]
        if par:
            cmd[1:1] = ["-fopenmp", "-D_GLIBCXX_PARALLEL"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def configure(lib: ctypes.CDLL) -> ctypes.CDLL:
    """Declare the C signatures on a loaded oracle library."""
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u64 = ctypes.c_uint64
    lib.oracle_sa.argtypes = [u8p, u64, u32p]
    lib.oracle_pd_names.argtypes = [u8p, u64, u64, u32p, u64p]
    lib.oracle_prefix_ranks.argtypes = [u8p, u64, u64, u32p]
    lib.oracle_brute_sa.argtypes = [u8p, u64, u32p]
    lib.oracle_check_sa.argtypes = [u8p, u64, u32p, u64p]
    lib.oracle_lcp.argtypes = [u8p, u64, u32p, u32p]
    lib.oracle_bwt.argtypes = [u8p, u64, u32p, u8p, u64p]
    lib.oracle_sa_interval.argtypes = [u8p, u64, u32p, u8p, u64, u64p, u64p]
    lib.oracle_pa_names.argtypes = [u8p, u64, ctypes.c_uint32, u64, u32p, u64p]
    lib.oracle_pa_sa.argtypes = [u8p, u64, ctypes.c_uint32, u32p]
    lib.oracle_opk_order.argtypes = [u64, u64, u32p]
    lib.oracle_pdd_sa.argtypes = [u8p, u64, u64, u32p, u64p, u64, u64p]
    lib.oracle_pdd_round.argtypes = [u8p, u64, u64, u64, u32p, u32p, u8p, u64p]
    lib.oracle_dc3_sample_ranks.argtypes = [u8p, u64, u32p, u32p]
    lib.oracle_dcx_sample_ranks.argtypes = [u8p, u64, ctypes.c_uint32, ctypes.c_uint32, u32p]
    for f in ("oracle_dc3_sample_ranks", "oracle_dcx_sample_ranks", "oracle_opk_order", "oracle_pdd_sa", "oracle_pdd_round","oracle_sa", "oracle_pd_names", "oracle_prefix_ranks", "oracle_pa_names",
              "oracle_pa_sa",
              "oracle_brute_sa", "oracle_check_sa", "oracle_num_threads",
              "oracle_lcp", "oracle_bwt", "oracle_sa_interval"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _lib(parallel: bool = False) -> ctypes.CDLL:
    with _lock:
        if parallel in _libs:
            return _libs[parallel]
        path = LIB_PAR if parallel else LIB_SEQ
        if not os.path.exists(path):
            build(parallel)
        _libs[parallel] = configure(ctypes.CDLL(path))
        return _libs[parallel]


def _text(t) -> np.ndarray:
    if isinstance(t, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(t), dtype=np.uint8)
    a = np.ascontiguousarray(t)
    if a.dtype != np.uint8:
        raise TypeError("text must be uint8")
    return a


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def sa(text, parallel: bool = False) -> np.ndarray:
    """Suffix array (uint32) by plain prefix doubling."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    rc = _lib(parallel).oracle_sa(_p(t, ctypes.c_uint8), t.size, _p(out, ctypes.c_uint32))
    if rc:
        raise ValueError("text too long for 32-bit suffix array")
    return out


def pd_names(text, steps: int) -> tuple[np.ndarray, int]:
    """Names after ``steps`` doubling sorts, and the prefix length they resolve."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    h = ctypes.c_uint64(0)
    rc = _lib().oracle_pd_names(_p(t, ctypes.c_uint8), t.size, steps,
                                _p(out, ctypes.c_uint32), ctypes.byref(h))
    if rc:
        raise ValueError("bad arguments")
    return out, int(h.value)


def pa_names(text, a: int, steps: int) -> tuple[np.ndarray, int]:
    """Names after at most ``steps`` sorts of a-tuples (prefix a-tupling; 0:
    the names of single characters), and the prefix length they resolve
    (a^steps, or the length at which every name became distinct)."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    h = ctypes.c_uint64(0)
    rc = _lib().oracle_pa_names(_p(t, ctypes.c_uint8), t.size, a, steps,
                                _p(out, ctypes.c_uint32), ctypes.byref(h))
    if rc:
        raise ValueError("bad arguments")
    return out, int(h.value)


def pa_sa(text, a: int) -> np.ndarray:
    """Suffix array by prefix a-tupling (a = 4: prefix quadrupling)."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    rc = _lib().oracle_pa_sa(_p(t, ctypes.c_uint8), t.size, a, _p(out, ctypes.c_uint32))
    if rc:
        raise ValueError("bad arguments")
    return out


def opk_order(n: int, h: int) -> np.ndarray:
    """Positions 0..n-1 ordered by (i mod h, i div h): the comparator of Eq. 1."""
    out = np.empty(n, dtype=np.uint32)
    if _lib().oracle_opk_order(n, h, _p(out, ctypes.c_uint32)):
        raise ValueError("bad arguments")
    return out


def pdd_sa(text, c: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """Suffix array by sort-based prefix doubling with discarding (Alg. 5) from
    names of c-character prefixes, and the per-round counts as rows
    (|P|, |I|, |D'|, |U'|): working items, non-unique items, items discarded
    (finalised), unique items kept for the next round."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    counts = np.zeros(4 * 64, dtype=np.uint64)
    rounds = ctypes.c_uint64(0)
    if _lib().oracle_pdd_sa(_p(t, ctypes.c_uint8), t.size, c, _p(out, ctypes.c_uint32),
                            _p(counts, ctypes.c_uint64), 64, ctypes.byref(rounds)):
        raise ValueError("bad arguments")
    r = int(rounds.value)
    return out, counts[:4 * r].reshape(r, 4)


def pdd_round(text, c: int, k: int):
    """The working items of round k (>= 1) of :func:`pdd_sa` after the
    comparator sort: (positions, names, unique flags), or None if the build
    ended before round k."""
    t = _text(text)
    n = t.size
    pos = np.empty(max(n, 1), dtype=np.uint32)
    names = np.empty(max(n, 1), dtype=np.uint32)
    uniq = np.empty(max(n, 1), dtype=np.uint8)
    m = ctypes.c_uint64(0)
    rc = _lib().oracle_pdd_round(_p(t, ctypes.c_uint8), n, c, k, _p(pos, ctypes.c_uint32),
                                 _p(names, ctypes.c_uint32), _p(uniq, ctypes.c_uint8),
                                 ctypes.byref(m))
    if rc:
        return None
    mm = int(m.value)
    return pos[:mm], names[:mm], uniq[:mm].astype(bool)


def dc3_sample_ranks(text) -> tuple[np.ndarray, np.ndarray]:
    """(R1, R2): 1-based ranks among all sample suffixes (positions i with
    i mod 3 != 0) of the suffixes 3t + 1 and 3t + 2."""
    t = _text(text)
    n = t.size
    r1 = np.zeros((n + 1) // 3, dtype=np.uint32)
    r2 = np.zeros(n // 3, dtype=np.uint32)
    if _lib().oracle_dc3_sample_ranks(_p(t, ctypes.c_uint8), n, _p(r1, ctypes.c_uint32),
                                      _p(r2, ctypes.c_uint32)):
        raise ValueError("bad arguments")
    return r1, r2


def dcx_sample_ranks(text, x: int, cover) -> np.ndarray:
    """Per position: the 1-based rank of the suffix among the suffixes starting
    at positions i with i mod x in ``cover``, 0 elsewhere."""
    t = _text(text)
    out = np.zeros(t.size, dtype=np.uint32)
    mask = 0
    for d in cover:
        mask |= 1 << int(d)
    if _lib().oracle_dcx_sample_ranks(_p(t, ctypes.c_uint8), t.size, x, mask,
                                      _p(out, ctypes.c_uint32)):
        raise ValueError("bad arguments")
    return out


def prefix_ranks(text, h: int) -> np.ndarray:
    """Closed-form names for prefix length ``h`` (1-based head ranks)."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    rc = _lib().oracle_prefix_ranks(_p(t, ctypes.c_uint8), t.size, h, _p(out, ctypes.c_uint32))
    if rc:
        raise ValueError("bad arguments")
    return out


def brute_sa(text) -> np.ndarray:
    """Suffix array straight from the definition (for small n)."""
    t = _text(text)
    out = np.empty(t.size, dtype=np.uint32)
    _lib().oracle_brute_sa(_p(t, ctypes.c_uint8), t.size, _p(out, ctypes.c_uint32))
    return out


def check_sa(text, sa_arr) -> tuple[int, int]:
    """Linear-time check. Returns (status, where): 0 ok, 1 not a permutation,
    2 adjacent-order violation at SA position ``where``."""
    t = _text(text)
    a = np.asarray(sa_arr)
    if a.dtype in (np.int32, np.uint32):
        s = np.ascontiguousarray(a).view(np.uint32)
    else:
        if a.size and (a.min() < 0 or a.max() >= 2**32):
            return 1, int(np.argmax((a < 0) | (a >= 2**32)))
        s = np.ascontiguousarray(a, dtype=np.uint32)
    if s.size != t.size:
        return 1, 0
    where = ctypes.c_uint64(0)
    rc = _lib().oracle_check_sa(_p(t, ctypes.c_uint8), t.size, _p(s, ctypes.c_uint32),
                                ctypes.byref(where))
    return int(rc), int(where.value)


def _sa32(text, sa_arr) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(sa_arr)).view(np.uint32) \
        if np.asarray(sa_arr).dtype in (np.int32, np.uint32) \
        else np.ascontiguousarray(sa_arr, dtype=np.uint32)
    if s.size != _text(text).size:
        raise ValueError("suffix array and text differ in length")
    return s


def lcp(text, sa_arr) -> np.ndarray:
    """LCP array of a text and its suffix array, by direct comparison of
    adjacent suffixes (uint32; lcp[0] = 0)."""
    t = _text(text)
    s = _sa32(t, sa_arr)
    out = np.empty(t.size, dtype=np.uint32)
    if _lib().oracle_lcp(_p(t, ctypes.c_uint8), t.size, _p(s, ctypes.c_uint32),
                         _p(out, ctypes.c_uint32)):
        raise ValueError("suffix array entry out of range")
    return out


def bwt(text, sa_arr) -> tuple[np.ndarray, int]:
    """Burrows-Wheeler transform of text$ from its suffix array: the n bytes of
    the transform without its $, and the row of the $."""
    t = _text(text)
    s = _sa32(t, sa_arr)
    out = np.empty(t.size, dtype=np.uint8)
    d = ctypes.c_uint64(0)
    if _lib().oracle_bwt(_p(t, ctypes.c_uint8), t.size, _p(s, ctypes.c_uint32),
                         _p(out, ctypes.c_uint8), ctypes.byref(d)):
        raise ValueError("suffix array entry out of range")
    return out, int(d.value)


def sa_interval(text, sa_arr, pattern) -> tuple[int, int]:
    """[lo, hi): the suffix-array positions whose suffixes start with pattern."""
    t = _text(text)
    s = _sa32(t, sa_arr)
    pt = _text(pattern)
    if pt.size == 0:
        pt = np.zeros(1, np.uint8)[:0]
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    buf = np.ascontiguousarray(pt) if pt.size else np.zeros(1, np.uint8)
    _lib().oracle_sa_interval(_p(t, ctypes.c_uint8), t.size, _p(s, ctypes.c_uint32),
                              _p(buf, ctypes.c_uint8), pt.size, ctypes.byref(lo),
                              ctypes.byref(hi))
    return int(lo.value), int(hi.value)


def num_threads(parallel: bool = True) -> int:
    return int(_lib(parallel).oracle_num_threads())
