"""Suffix-array construction on MI355X (gfx950) by prefix doubling with discarding.

Python face of the HIP library ``libsa_mi355x.so`` (C ABI in include/sa.h).
Texts and suffix arrays are PyTorch CUDA tensors; every step runs in the
library's kernels on the tensor's device and the current stream.

    >>> from paper_1610_03007_amd import SuffixArrayBuilder
    >>> b = SuffixArrayBuilder()
    >>> sa = b.build(torch.frombuffer(bytearray(b"banana"), dtype=torch.uint8).cuda())
    >>> sa.tolist()
    [5, 3, 1, 0, 4, 2]
"""

from __future__ import annotations

import ctypes
import os

import torch

from . import _native
from ._native import SAError, check

__all__ = ["SuffixArrayBuilder", "SuffixArrayServer", "FMIndex", "SAError", "workspace_bytes"]


# Tuning cache shipped with the package: entries found by the autotuner on
# MI355X for the standard workload sizes. Builders use it unless told otherwise.
DEFAULT_TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_bytes(total_n: int, num_texts: int = 1) -> int:
    """Device workspace (bytes) a build of ``num_texts`` texts of ``total_n``
    bytes in all needs (one text: ``sa_build``; more: ``sa_build_batch``)."""
    return int(_native.lib().sa_workspace_bytes(total_n, num_texts))


class SuffixArrayBuilder:
    """Owns a library context (device workspace, kernel statistics) on one GPU.

    ``tune_cache``: path of a tuning cache (JSON); None takes the package's
    cache when present, "" none (library defaults)."""

    def __init__(self, device: int | torch.device | None = None, tune_cache: str | None = None):
        if tune_cache is None:
            tune_cache = DEFAULT_TUNE_CACHE if os.path.exists(DEFAULT_TUNE_CACHE) else ""
        self.tune_cache = tune_cache or None
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device if isinstance(device, int) else device.index)
        self._lib = _native.lib()
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self._lib.sa_ctx_create(ctypes.byref(self._ctx), self.device.index,
                                          tune_cache.encode() if tune_cache else None),
                  "sa_ctx_create")

    def close(self) -> None:
        if self._ctx:
            self._lib.sa_ctx_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover - interpreter shutdown order varies
        try:
            self.close()
        except Exception:
            pass

    def _text(self, text: torch.Tensor) -> torch.Tensor:
        if not isinstance(text, torch.Tensor) or text.dtype != torch.uint8:
            raise TypeError("text must be a torch.uint8 tensor")
        if text.device != self.device:
            raise ValueError(f"text is on {text.device}, builder on {self.device}")
        return text.contiguous().view(-1)

    def _out(self, out: torch.Tensor | None, n: int, name: str) -> torch.Tensor:
        if out is None:
            return torch.empty(n, dtype=torch.int32, device=self.device)
        if out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() \
                or out.device != self.device:
            raise ValueError(f"{name} must be a contiguous int32 tensor of {n} elements on "
                             f"{self.device}")
        return out

    def build(self, text: torch.Tensor, out: torch.Tensor | None = None,
              sigma: int = 256) -> torch.Tensor:
        """Suffix array of ``text`` as int32 (values < n, bit pattern of the u32 SA)."""
        t = self._text(text)
        n = t.numel()
        sa = self._out(out, n, "out")
        with torch.cuda.device(self.device):
            check(self._lib.sa_build(self._ctx, ctypes.c_void_p(t.data_ptr()), n, sigma,
                                     ctypes.c_void_p(sa.data_ptr()), _stream_handle(self.device)),
                  "sa_build")
        return sa

    def build_sorted_pairs(self, text: torch.Tensor, out: torch.Tensor | None = None,
                           sigma: int = 256):
        """Suffix array by prefix doubling with discarding by sorting (no inverse
        suffix array; ``sa_build_sorted_pairs``). Returns (sa, counts): counts
        is a (rounds, 4) uint64 array of |P|, |I|, discarded, kept per round."""
        import numpy as np
        t = self._text(text)
        n = t.numel()
        sa = self._out(out, n, "out")
        counts = np.zeros((64, 4), dtype=np.uint64)
        with torch.cuda.device(self.device):
            check(self._lib.sa_build_sorted_pairs(
                self._ctx, ctypes.c_void_p(t.data_ptr()), n, sigma,
                ctypes.c_void_p(sa.data_ptr()), counts.ctypes.data_as(ctypes.c_void_p), 64,
                _stream_handle(self.device)), "sa_build_sorted_pairs")
        rounds = self.last_info()["rounds"] if n else 1
        return sa, counts[:max(0, rounds - 1)]

    def build_dc3(self, text: torch.Tensor, out: torch.Tensor | None = None,
                  with_ranks: bool = False):
        """Suffix array by DC3 (``sa_build_dc3``). With ``with_ranks`` returns
        (sa, rank12): the top level's sample ranks by position (0 at positions
        divisible by 3)."""
        t = self._text(text)
        n = t.numel()
        sa = self._out(out, n, "out")
        r12 = torch.empty(n, dtype=torch.int32, device=self.device) if with_ranks else None
        with torch.cuda.device(self.device):
            check(self._lib.sa_build_dc3(self._ctx, ctypes.c_void_p(t.data_ptr()), n,
                                         ctypes.c_void_p(sa.data_ptr()),
                                         ctypes.c_void_p(r12.data_ptr() if r12 is not None
                                                         else None),
                                         _stream_handle(self.device)), "sa_build_dc3")
        return (sa, r12) if with_ranks else sa

    def build_dc7(self, text: torch.Tensor, out: torch.Tensor | None = None,
                  with_ranks: bool = False):
        """Suffix array by DC7 (``sa_build_dc7``). With ``with_ranks`` returns
        (sa, ranks): the sample ranks by position (0 outside the sample)."""
        t = self._text(text)
        n = t.numel()
        sa = self._out(out, n, "out")
        rk = torch.empty(n, dtype=torch.int32, device=self.device) if with_ranks else None
        with torch.cuda.device(self.device):
            check(self._lib.sa_build_dc7(self._ctx, ctypes.c_void_p(t.data_ptr()), n,
                                         ctypes.c_void_p(sa.data_ptr()),
                                         ctypes.c_void_p(rk.data_ptr() if rk is not None
                                                         else None),
                                         _stream_handle(self.device)), "sa_build_dc7")
        return (sa, rk) if with_ranks else sa

    def build_batch(self, texts: torch.Tensor, offsets, out: torch.Tensor | None = None):
        """Suffix arrays of many texts in one batched build.

        ``texts``: uint8 CUDA tensor, the texts concatenated; ``offsets``: the
        num_texts + 1 boundaries (any integer sequence or array, host side).
        Returns an int32 tensor aligned with ``texts`` holding each text's
        suffix array (local positions) at that text's slice."""
        import numpy as np
        t = self._text(texts)
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        if off.ndim != 1 or off.size < 2:
            raise ValueError("offsets must hold num_texts + 1 boundaries")
        if int(off[-1]) != t.numel():
            raise ValueError("offsets[-1] must equal the total text length")
        sa = self._out(out, t.numel(), "out")
        with torch.cuda.device(self.device):
            check(self._lib.sa_build_batch(self._ctx, ctypes.c_void_p(t.data_ptr()),
                                           off.ctypes.data_as(ctypes.c_void_p), off.size - 1,
                                           ctypes.c_void_p(sa.data_ptr()),
                                           _stream_handle(self.device)), "sa_build_batch")
        return sa

    def build_rounds(self, text: torch.Tensor, max_rounds: int):
        """Run at most ``max_rounds`` doubling rounds. Returns (sa, isa, info):
        the partially finalised SA, the names after the last round run, and the
        build diagnostics (``info['prefix_len']`` is the prefix length the names
        resolve)."""
        t = self._text(text)
        n = t.numel()
        sa = torch.zeros(n, dtype=torch.int32, device=self.device)
        isa = torch.zeros(n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            check(self._lib.sa_build_rounds(self._ctx, ctypes.c_void_p(t.data_ptr()), n,
                                            max_rounds, ctypes.c_void_p(sa.data_ptr()),
                                            ctypes.c_void_p(isa.data_ptr()),
                                            _stream_handle(self.device)), "sa_build_rounds")
        return sa, isa, self.last_info()

    def radix_sort_pairs(self, keys: torch.Tensor, vals: torch.Tensor, key_bits: int = 64):
        """Stable sort of (int64 key bits as u64, int32 value bits as u32) pairs
        in place by the low ``key_bits`` bits of the key."""
        if keys.dtype != torch.int64 or vals.dtype != torch.int32:
            raise TypeError("keys must be int64 and vals int32 tensors")
        if keys.numel() != vals.numel() or not keys.is_contiguous() or not vals.is_contiguous():
            raise ValueError("keys and vals must be contiguous and of equal length")
        with torch.cuda.device(self.device):
            check(self._lib.sa_radix_sort_pairs(self._ctx, ctypes.c_void_p(keys.data_ptr()),
                                                ctypes.c_void_p(vals.data_ptr()), keys.numel(),
                                                key_bits, _stream_handle(self.device)),
                  "sa_radix_sort_pairs")
        return keys, vals

    def _sa_of(self, sa: torch.Tensor, n: int) -> torch.Tensor:
        if sa.dtype not in (torch.int32, torch.uint32) or sa.numel() != n \
                or not sa.is_contiguous() or sa.device != self.device:
            raise ValueError(f"sa must be a contiguous 32-bit tensor of {n} elements on "
                             f"{self.device}")
        return sa

    def lcp(self, text: torch.Tensor, sa: torch.Tensor,
            out: torch.Tensor | None = None) -> torch.Tensor:
        """LCP array (int32 bits of u32) of ``text`` and its suffix array ``sa``:
        out[0] = 0, out[j] = common prefix length of suffixes sa[j-1] and sa[j]."""
        t = self._text(text)
        n = t.numel()
        s = self._sa_of(sa, n)
        lcp = self._out(out, n, "out")
        with torch.cuda.device(self.device):
            check(self._lib.sa_lcp(self._ctx, ctypes.c_void_p(t.data_ptr()), n,
                                   ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(lcp.data_ptr()),
                                   _stream_handle(self.device)), "sa_lcp")
        return lcp

    def bwt(self, text: torch.Tensor, sa: torch.Tensor):
        """Burrows-Wheeler transform of text$: (uint8 tensor of n bytes without
        the $, row of the $)."""
        t = self._text(text)
        n = t.numel()
        s = self._sa_of(sa, n)
        out = torch.empty(n, dtype=torch.uint8, device=self.device)
        d = ctypes.c_uint64(0)
        with torch.cuda.device(self.device):
            check(self._lib.sa_bwt(self._ctx, ctypes.c_void_p(t.data_ptr()), n,
                                   ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.byref(d), _stream_handle(self.device)), "sa_bwt")
        return out, int(d.value)

    def fm_index(self, text: torch.Tensor, sa: torch.Tensor) -> "FMIndex":
        """FM index of ``text`` (device memory owned by the returned object)."""
        return FMIndex(self, text, sa)

    def last_info(self) -> dict:
        info = _native.BuildInfo()
        check(self._lib.sa_last_build_info(self._ctx, ctypes.byref(info)), "sa_last_build_info")
        return info.as_dict()

    def set_isa_mode(self, mode: str = "auto") -> None:
        """'auto', 'eager' or 'lazy' inverse-suffix-array formation after round 0."""
        check(self._lib.sa_ctx_set_isa_mode(self._ctx, _native.ISA_MODES[mode]),
              "sa_ctx_set_isa_mode")

    def tuning(self) -> dict:
        """The knobs of the last build (or the explicit tuning, or the defaults)."""
        t = _native.Tuning()
        check(self._lib.sa_ctx_get_tuning(self._ctx, ctypes.byref(t)), "sa_ctx_get_tuning")
        return _native.tuning_dict(t)

    def tuning_source(self) -> str:
        """Where the last build's knobs came from: 'default', 'cache' or 'explicit'."""
        v = ctypes.c_int(0)
        check(self._lib.sa_ctx_tuning_source(self._ctx, ctypes.byref(v)), "sa_ctx_tuning_source")
        return ("default", "cache", "explicit")[v.value]

    def set_tuning(self, **kw) -> None:
        """Set tuning knobs (sort_items, sort_block, sort_match, lazy_ratio,
        round0_full, sort_wgs_per_cu); results never change. Unset knobs keep
        their current values."""
        cur = self.tuning()
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning knobs {sorted(unknown)}")
        cur.update(kw)
        t = _native.Tuning(**cur)
        check(self._lib.sa_ctx_set_tuning(self._ctx, ctypes.byref(t)), "sa_ctx_set_tuning")

    def auto_tuning(self) -> None:
        """Drop an explicit tuning: builds take the cache entry for their input,
        else the defaults."""
        check(self._lib.sa_ctx_set_tuning(self._ctx, None), "sa_ctx_set_tuning")

    def tune(self, texts: torch.Tensor, offsets=None, reps: int = 3):
        """Autotune on this input (one text, or a batch with ``offsets``): records
        the fastest tuning in the context's cache table and returns
        (tuning dict, best build ms). ``save_tuning`` writes the table."""
        import numpy as np
        t = self._text(texts)
        off = np.ascontiguousarray(np.asarray([0, t.numel()] if offsets is None else offsets,
                                              dtype=np.uint64))
        if off.ndim != 1 or off.size < 2 or int(off[-1]) != t.numel():
            raise ValueError("offsets must hold num_texts + 1 boundaries ending at the length")
        sa = torch.empty(t.numel(), dtype=torch.int32, device=self.device)
        best = _native.Tuning()
        ms = ctypes.c_double(0)
        with torch.cuda.device(self.device):
            check(self._lib.sa_tune(self._ctx, ctypes.c_void_p(t.data_ptr()),
                                    off.ctypes.data_as(ctypes.c_void_p), off.size - 1,
                                    ctypes.c_void_p(sa.data_ptr()), _stream_handle(self.device),
                                    reps, ctypes.byref(best), ctypes.byref(ms)), "sa_tune")
        return _native.tuning_dict(best), float(ms.value)

    def save_tuning(self, path: str | None = None) -> None:
        """Write the cache table as JSON (default: the tune_cache path)."""
        check(self._lib.sa_tune_save(self._ctx, path.encode() if path else None), "sa_tune_save")

    def set_trace(self, on: bool = True) -> None:
        check(self._lib.sa_ctx_set_trace(self._ctx, 1 if on else 0), "sa_ctx_set_trace")

    def reset_stats(self) -> None:
        check(self._lib.sa_ctx_reset_stats(self._ctx), "sa_ctx_reset_stats")

    def kernel_stats(self) -> dict:
        out = {}
        for name, kind in _native.KERNEL_KINDS.items():
            st = _native.KernelStats()
            check(self._lib.sa_ctx_get_kernel_stats(self._ctx, kind, ctypes.byref(st)),
                  "sa_ctx_get_kernel_stats")
            out[name] = {"launches": int(st.launches), "ms": float(st.ms), "bytes": float(st.bytes)}
        return out


class SuffixArrayServer:
    """Continuous-batching suffix-array service on one GPU (sa_server_* ABI).

    ``submit`` queues a host text and returns a ticket; the library's worker
    thread admits requests as slots and device memory free up and runs merged
    doubling rounds over all admitted requests. ``poll`` returns the suffix
    array once it is complete, with the submit-to-ready latency."""

    def __init__(self, device: int = 0, capacity_bytes: int = 0, max_text: int = 0):
        self._lib = _native.lib()
        self._srv = ctypes.c_void_p()
        self.device = device
        with torch.cuda.device(device):
            check(self._lib.sa_server_create(ctypes.byref(self._srv), device, capacity_bytes,
                                             max_text), "sa_server_create")
        self._n = {}

    def close(self) -> None:
        if self._srv:
            self._lib.sa_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def submit(self, text) -> int:
        import numpy as np
        a = np.ascontiguousarray(np.frombuffer(bytes(text), np.uint8)
                                 if isinstance(text, (bytes, bytearray)) else text, dtype=np.uint8)
        t = ctypes.c_uint64()
        check(self._lib.sa_server_submit(self._srv, a.ctypes.data_as(ctypes.c_void_p), a.size,
                                         ctypes.byref(t)), "sa_server_submit")
        self._n[t.value] = a.size
        return int(t.value)

    def poll(self, ticket: int, out=None):
        """(done, suffix array or None, latency in ms or None).

        Without ``out`` the array comes back as numpy uint32 over pinned host
        memory (one direct copy from the device). ``out`` may instead be a
        contiguous 32-bit torch tensor of the text's length, in host or device
        memory, which is filled and returned."""
        import numpy as np
        n = self._n[ticket]
        done = ctypes.c_int(0)
        lat = ctypes.c_double(0.0)
        if n:
            # Ask first without a buffer (cheap while the request is running).
            check(self._lib.sa_server_poll(self._srv, ticket, None, ctypes.byref(done), None),
                  "sa_server_poll")
            if done.value != 2:
                return False, None, None
        if out is None:
            buf = torch.empty(n, dtype=torch.int32, pin_memory=n > 0)
            res = buf.numpy().view(np.uint32)
        else:
            if not (isinstance(out, torch.Tensor) and out.is_contiguous()
                    and out.dtype in (torch.int32, torch.uint32) and out.numel() == n):
                raise ValueError("out must be a contiguous 32-bit tensor of the text's length")
            buf = res = out
        ptr = ctypes.c_void_p(buf.data_ptr()) if n else None
        check(self._lib.sa_server_poll(self._srv, ticket, ptr, ctypes.byref(done),
                                       ctypes.byref(lat)), "sa_server_poll")
        if done.value != 1:
            return False, None, None
        del self._n[ticket]
        return True, res, float(lat.value)

    def stats(self) -> dict:
        st = _native.ServerStats()
        check(self._lib.sa_server_stats(self._srv, ctypes.byref(st)), "sa_server_stats")
        return {k: getattr(st, k) for k, _ in _native.ServerStats._fields_}


class FMIndex:
    """FM index on the GPU (sa_fm_* ABI): pattern queries by backward search.

    ``count(patterns)`` takes a list of bytes-like patterns (or a uint8 CUDA
    tensor of the patterns concatenated plus host offsets) and returns an int64
    tensor of shape (num, 2): for each pattern the suffix-array positions
    [lo, hi) whose suffixes start with it."""

    def __init__(self, builder: SuffixArrayBuilder, text: torch.Tensor, sa: torch.Tensor):
        t = builder._text(text)
        n = t.numel()
        s = builder._sa_of(sa, n)
        self.device = builder.device
        self._lib = builder._lib
        self._fm = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self._lib.sa_fm_create(ctypes.byref(self._fm), builder._ctx,
                                         ctypes.c_void_p(t.data_ptr()), n,
                                         ctypes.c_void_p(s.data_ptr()),
                                         _stream_handle(self.device)), "sa_fm_create")

    def info(self) -> dict:
        n, d, b = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        sg = ctypes.c_uint32()
        check(self._lib.sa_fm_info(self._fm, ctypes.byref(n), ctypes.byref(d), ctypes.byref(sg),
                                   ctypes.byref(b)), "sa_fm_info")
        return {"n": n.value, "dollar": d.value, "sigma": sg.value, "device_bytes": b.value}

    def count(self, patterns, offsets=None) -> torch.Tensor:
        import numpy as np
        if offsets is None:
            pats = [bytes(p) for p in patterns]
            off = np.zeros(len(pats) + 1, dtype=np.uint64)
            np.cumsum([len(p) for p in pats], out=off[1:])
            cat = b"".join(pats)
            data = torch.frombuffer(bytearray(cat), dtype=torch.uint8).to(self.device) \
                if cat else torch.zeros(1, dtype=torch.uint8, device=self.device)
        else:
            data = patterns
            off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        num = off.size - 1
        d_off = torch.from_numpy(off.view(np.int64)).to(self.device)
        ranges = torch.empty((num, 2), dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            check(self._lib.sa_fm_count(self._fm, ctypes.c_void_p(data.data_ptr()),
                                        ctypes.c_void_p(d_off.data_ptr()), num,
                                        ctypes.c_void_p(ranges.data_ptr()),
                                        _stream_handle(self.device)), "sa_fm_count")
        return ranges

    def close(self) -> None:
        if self._fm:
            self._lib.sa_fm_destroy(self._fm)
            self._fm = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
