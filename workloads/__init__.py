"""Seeded synthetic workloads (inputs only; no suffix-sorting arithmetic).

The same generators feed the CPU oracle and the HIP library in the tests and the
benchmark. Each workload stands in for a class of real text:

* :func:`dna` -- iid uniform over ``ACGT`` (2 bits/symbol, every short k-mer repeats).
* :func:`markov3` -- order-3 Markov chain over 96 printable bytes (``\\n`` and
  0x20..0x7E); each of the 96^3 context rows is drawn from Dirichlet(0.1).
* :func:`repetitive` -- a 256 KiB iid base string over the same 96 symbols,
  concatenated 4096 times, each byte of each copy independently replaced with
  probability 1e-4 by a uniformly chosen different symbol (long common prefixes).
* :func:`batch` -- thousands of texts with log-uniform lengths, alternating DNA
  and Markov texts, concatenated with CSR offsets.

DNA, repetitive and batch-length draws use numpy's PCG64 (``default_rng(seed)``);
the Markov table and chains come from ``gen.c`` (xoshiro256** seeded with
SplitMix64, Marsaglia-Tsang gamma variates, 16-bit cumulative thresholds).
"""

from __future__ import annotations

import concurrent.futures as cf
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
LIB = os.path.join(_HERE, "libgen.so")

MARKOV_K = 96
MARKOV_ALPHA = 0.1
SYMBOLS96 = np.array([0x0A] + list(range(0x20, 0x7F)), dtype=np.uint8)
assert SYMBOLS96.size == MARKOV_K

_lock = threading.Lock()
_lib = None
_cdf_cache: dict[int, np.ndarray] = {}


def build() -> None:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            lib = ctypes.CDLL(LIB)
            lib.gen_markov3.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64]
            lib.gen_markov3.restype = None
            lib.gen_markov_table.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_void_p]
            lib.gen_markov_table.restype = None
            _lib = lib
        return _lib


def dna(n: int, seed: int = 0) -> np.ndarray:
    """n bytes iid uniform over ACGT."""
    return np.frombuffer(b"ACGT", dtype=np.uint8)[np.random.default_rng(seed).integers(0, 4, n)]


def markov_table(matrix_seed: int = 1) -> np.ndarray:
    """16-bit cumulative transition table, shape (96^3, 95); rows ~ Dirichlet(0.1)."""
    with _lock:
        if matrix_seed in _cdf_cache:
            return _cdf_cache[matrix_seed]
    tab = np.empty((MARKOV_K ** 3, MARKOV_K - 1), dtype=np.uint16)
    _load().gen_markov_table(matrix_seed, MARKOV_K, 3, MARKOV_ALPHA, tab.ctypes.data)
    with _lock:
        _cdf_cache[matrix_seed] = tab
    return tab


def markov3_many(lengths, seeds, matrix_seed: int = 1,
                 burn_in: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """Several independent Markov texts, concatenated. Returns (bytes, offsets)."""
    lengths = np.asarray(lengths, dtype=np.uint64)
    seeds = np.asarray(seeds, dtype=np.uint64)
    offsets = np.zeros(lengths.size + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    out = np.empty(int(offsets[-1]), dtype=np.uint8)
    if out.size:
        cdf = markov_table(matrix_seed)
        _load().gen_markov3(cdf.ctypes.data, MARKOV_K, SYMBOLS96.ctypes.data, out.ctypes.data,
                            offsets.ctypes.data, lengths.ctypes.data, seeds.ctypes.data,
                            lengths.size, burn_in)
    return out, offsets


MARKOV_SEGMENT = 1 << 22
MARKOV_BURN_IN = 4096


def markov3(n: int, chain_seed: int = 2, matrix_seed: int = 1) -> np.ndarray:
    """n bytes of the order-3 Markov source.

    Up to 4 MiB this is one chain started from context (0, 0, 0) with seed
    ``chain_seed``. Longer texts are 4 MiB segments, segment s drawn from its own
    chain (seed ``chain_seed * 2^20 + s``, 4096 burn-in steps dropped) so that
    they can be generated in parallel; the joins are the only places where the
    text is not one continuous chain.
    """
    if n <= MARKOV_SEGMENT:
        return markov3_many([n], [chain_seed], matrix_seed)[0]
    nseg = (n + MARKOV_SEGMENT - 1) // MARKOV_SEGMENT
    lengths = [MARKOV_SEGMENT] * (nseg - 1) + [n - MARKOV_SEGMENT * (nseg - 1)]
    seeds = [(chain_seed << 20) + s for s in range(nseg)]
    return markov3_many(lengths, seeds, matrix_seed, MARKOV_BURN_IN)[0]


def repetitive(copies: int = 4096, base_len: int = 262144, p: float = 1e-4,
               base_seed: int = 3, sub_seed: int = 4) -> np.ndarray:
    """``copies`` copies of a random base string with rate-``p`` substitutions."""
    base_idx = np.random.default_rng(base_seed).integers(0, MARKOV_K, base_len).astype(np.uint8)
    idx = np.tile(base_idx, copies)
    n = idx.size
    rng = np.random.default_rng(sub_seed)
    # Independent Bernoulli(p) per position == geometric gaps between hits.
    est = int(n * p * 1.2) + 64
    pos = []
    last = -1
    while True:
        gaps = rng.geometric(p, size=est)
        cand = last + np.cumsum(gaps)
        keep = cand[cand < n]
        pos.append(keep)
        if keep.size < cand.size:
            break
        last = int(cand[-1])
    pos = np.concatenate(pos).astype(np.int64)
    shift = rng.integers(1, MARKOV_K, pos.size).astype(np.uint8)
    idx[pos] = ((idx[pos].astype(np.int64) + shift) % MARKOV_K).astype(np.uint8)
    return SYMBOLS96[idx]


def batch_lengths(num_texts: int = 4096, lo: int = 4096, hi: int = 8388608,
                  seed: int = 5) -> np.ndarray:
    u = np.random.default_rng(seed).uniform(np.log(lo), np.log(hi), num_texts)
    return np.floor(np.exp(u)).astype(np.int64)


def batch(num_texts: int = 4096, lo: int = 4096, hi: int = 8388608, seed: int = 5,
          matrix_seed: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Concatenated texts and CSR offsets (uint64, length num_texts + 1).
    Even t: DNA with seed 1000 + t; odd t: Markov chain with seed 2000 + t."""
    lengths = batch_lengths(num_texts, lo, hi, seed)
    offsets = np.zeros(num_texts + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    out = np.empty(int(offsets[-1]), dtype=np.uint8)
    odd = np.arange(1, num_texts, 2)
    if odd.size:
        mk, mk_off = markov3_many(lengths[odd], 2000 + odd, matrix_seed)
        for j, t in enumerate(odd):
            out[offsets[t]:offsets[t + 1]] = mk[mk_off[j]:mk_off[j + 1]]
    def fill_dna(t: int) -> None:
        out[offsets[t]:offsets[t + 1]] = dna(int(lengths[t]), 1000 + t)

    # numpy draws without holding the interpreter lock: texts in parallel.
    with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(fill_dna, range(0, num_texts, 2)))
    return out, offsets


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


DNA_CHUNK = 1 << 24


def dna_long(n: int, seed: int = 0) -> np.ndarray:
    """n bytes iid uniform over ACGT, drawn in 16 MiB chunks: chunk k from
    ``default_rng(seed * 2^20 + k)`` (chunks generated in parallel)."""
    out = np.empty(n, dtype=np.uint8)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)

    def fill(k: int) -> None:
        a = k * DNA_CHUNK
        b = min(n, a + DNA_CHUNK)
        out[a:b] = acgt[np.random.default_rng((seed << 20) + k).integers(0, 4, b - a)]

    with cf.ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(fill, range((n + DNA_CHUNK - 1) // DNA_CHUNK)))
    return out
