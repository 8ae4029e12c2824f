#!/usr/bin/env python3
"""Benchmark: suffix-array construction on one MI355X.

The default run measures every workload of the suffix-array hot path and prints
one JSON line. Its headline (``value``) is the largest single-GPU workload: one
batched build of 4096 texts (4.46e9 bytes in all). One step is one complete
``sa_build_batch`` (every doubling round: key packing, radix sort, re-rank / ISA
scatter / discard) with the texts already resident in HBM. ``configs`` carries
a record per workload:

* ``batch_4096`` -- batched vs per-text (one ``sa_build`` per text, same GPU);
* ``repetitive_1g``, ``markov_256m``, ``dna_1m`` -- one text per ``sa_build``;
* ``serve`` -- a Poisson request stream through the continuous-batching server
  and through one ``sa_build`` per request: p50/p99 latency, sustained
  throughput, and capacity with a burst of requests.

Every build record has Msuffixes/s, the whole-build HBM roofline (algorithmic
bytes of the method over the build time, against 8 TB/s), the radix-sort sweep's
roofline from HIP events around each launch, a per-kernel table, and the CPU
oracle (plain prefix doubling) timed on a bounded sample at one thread and on
all host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|NAME]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "Msuffixes/s on 1 GPU + HBM roofline %; batched vs per-text; p50/p99 latency"
WORKLOADS = {
    "batch_4096": "4096 texts, lengths log-uniform in [4 KiB, 8 MiB], half ACGT, half "
                  "order-3 Markov (96 bytes); one batched build",
    "repetitive_1g": "256 KiB base x 4096 copies, 1e-4 substitutions, n=2^30",
    "markov_256m": "order-3 Markov text, 96 printable bytes, Dirichlet(0.1) rows, n=2^28",
    "dna_1m": "uniform ACGT text, seed 0, n=2^20",
    "serve": "Poisson arrivals at 330.5 req/s (2 GB/s of text), lengths log-uniform in "
             "[1 KiB, 64 MiB], ACGT or Markov slices; continuous-batching server",
}
BUILD_ORDER = ("batch_4096", "repetitive_1g", "markov_256m", "dna_1m")
SERVE_RATE = 330.5
SERVE_LO, SERVE_HI = 1024, 1 << 26
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_03007_amd", "csrc", "sa_kernels.hip")

# Bounded CPU-oracle samples (bytes): (one thread, all cores).
CPU_SAMPLES = {
    "batch_4096": (1 << 24, 1 << 26),
    "repetitive_1g": (1 << 23, 1 << 25),
    "markov_256m": (1 << 24, 1 << 28),
    "dna_1m": (1 << 20, 1 << 20),
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_text(name: str):
    """Returns (text, offsets or None)."""
    import workloads as W
    if name == "batch_4096":
        return W.batch()
    if name == "markov_256m":
        return W.markov3(1 << 28, chain_seed=2), None
    if name == "dna_1m":
        return W.dna(1 << 20, seed=0), None
    if name == "repetitive_1g":
        return W.repetitive(), None
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash() -> str:
    """sha256[:16] of the sort sweep's source: common.h, sa_kernels.hip from its
    top through the helper namespace (digit extraction, scans, look-back), and
    the sweep kernel from its leading comment to onesweep_supported."""
    with open(KERNEL_SOURCE) as f:
        src = f.read()
    with open(os.path.join(os.path.dirname(KERNEL_SOURCE), "common.h")) as f:
        common = f.read()
    head = src[:src.index("}  // namespace")]
    sweep = src[src.index("// One stable counting sweep over digit"):src.index("bool onesweep_supported(")]
    return hashlib.sha256((common + head + sweep).encode()).hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per sort-sweep launch from committed rocprofv3 counter runs,
    or None when absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def algorithmic_bytes(info: dict) -> float:
    """Bytes the method must move for one build (whole-build roofline):
    13 per suffix for the round-0 keys (text, key, value), 4 per suffix for the
    SA, and per round k with A_k suffixes sorted in P_k radix passes:
    A_k * (24 P_k + 24) (sweeps, the up-front histogram and the re-rank),
    24 A_k for the pair build (k >= 1) and 8 A_{k+1} for the survivors. A dense
    round (every suffix, names read in position order) builds its keys from 16
    bytes per suffix and its first sweep generates the values (4 fewer)."""
    A, P, n = info["active"], info["passes_run"], info["n"]
    dense = set(info.get("dense_rounds", []))
    b = 17.0 * n
    for k, a in enumerate(A):
        b += a * (24.0 * P[k] + 24.0)
        if k >= 1:
            b += (12.0 if k in dense else 24.0) * a
        if k + 1 < len(A):
            b += 8.0 * A[k + 1]
    return b


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_oracle(text, offsets, sample: int, parallel: bool) -> dict:
    """The CPU oracle on the first `sample` bytes (one text) or on whole texts
    of a batch in order until `sample` bytes."""
    import oracle
    if offsets is None:
        s = text[:sample].copy()
        t0 = time.perf_counter()
        oracle.sa(s, parallel=parallel)
        dt = time.perf_counter() - t0
        total, what = s.size, f"first {s.size} bytes of the text"
    else:
        t0 = time.perf_counter()
        total = ntexts = 0
        for t in range(offsets.size - 1):
            a, b = int(offsets[t]), int(offsets[t + 1])
            oracle.sa(text[a:b], parallel=parallel)
            total += b - a
            ntexts += 1
            if total >= sample:
                break
        dt = time.perf_counter() - t0
        what = f"the first {ntexts} texts of the batch ({total} bytes), one oracle call per text"
    return {
        "value": round(total / dt / 1e6, 3),
        "unit": "Msuffixes/s",
        "cores": oracle.num_threads(parallel=parallel),
        "kind": "oracle",
        "sample": f"{what}; plain prefix doubling, "
                  f"{'GNU parallel std::sort' if parallel else 'std::sort, one thread'}; "
                  f"{dt:.2f} s",
    }


def cpu_rows(name: str, text, offsets) -> dict:
    one, alln = CPU_SAMPLES[name]
    log(f"{name}: CPU oracle, one thread on {one} bytes, all cores on {alln} bytes")
    par = time_oracle(text, offsets, min(alln, text.size), parallel=True)
    seq = time_oracle(text, offsets, min(one, text.size), parallel=False)
    par["single_thread"] = seq
    par["cpu_model"] = cpu_model()
    par["nproc"] = os.cpu_count()
    return par


def kernel_table(stats: dict, steps: int) -> dict:
    out = {}
    for k, v in stats.items():
        if v["launches"] == 0:
            continue
        gbs = v["bytes"] / (v["ms"] / 1e3) / 1e9 if v["ms"] > 0 else 0.0
        out[k] = {"ms_per_step": round(v["ms"] / steps, 4), "launches": v["launches"],
                  "gb_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def run_build(name: str, steps: int, warmup: int, cpu: bool, sort_items: int = 0,
              per_text: bool = True) -> dict:
    """Times `steps` builds of one workload (HIP events on the build stream)."""
    import torch

    from paper_1610_03007_amd import SuffixArrayBuilder

    t_gen = time.perf_counter()
    text, offsets = make_text(name)
    n = int(text.size)
    log(f"{name}: n={n} generated in {time.perf_counter() - t_gen:.1f}s")
    dev = torch.device("cuda", 0)
    d_text = torch.from_numpy(text).to(dev)
    d_sa = torch.empty(n, dtype=torch.int32, device=dev)
    b = SuffixArrayBuilder(0)
    if sort_items:
        b.set_tuning(sort_items=sort_items)

    def step():
        if offsets is None:
            b.build(d_text, out=d_sa)
        else:
            b.build_batch(d_text, offsets, out=d_sa)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)

    def timed(trace: bool):
        b.reset_stats()
        b.set_trace(trace)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        b.set_trace(False)
        return e0.elapsed_time(e1), time.perf_counter() - t0

    # The timed steps run the product path: later rounds enqueued ahead of the
    # host and replayed from captured graphs. Per-kernel HIP events need every
    # kernel launched directly (one round per readback), so the kernel table
    # and the sweep roofline come from the same number of traced steps after.
    gpu_ms, wall = timed(False)
    info = b.last_info()
    traced_ms, _ = timed(True)
    stats = b.kernel_stats()
    ms = gpu_ms / steps
    value = n / (ms / 1e3) / 1e6
    balg = algorithmic_bytes(info)
    whole = balg / (ms / 1e3) / 1e9
    sweep = stats["sort_pass"]
    achieved = sweep["bytes"] / (sweep["ms"] / 1e3) / 1e9 if sweep["ms"] > 0 else 0.0
    rec = {
        "workload": name,
        "description": WORKLOADS[name],
        "n": n,
        "steps": steps,
        "warmup": warmup,
        "ms_per_build": round(ms, 4),
        "msuffixes_s": round(value, 2),
        "traced_ms_per_build": round(traced_ms / steps, 4),
        "graph_rounds_last_build": info["graph_rounds"],
        "whole_build_roofline": {
            "bound": "hbm", "algorithmic_bytes": round(balg), "achieved": round(whole, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(whole / HBM_PEAK_GBS, 4)},
        "sweep_roofline": {
            "bound": "hbm", "kernel": "onesweep_pass_kernel", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name),
            "algorithmic_bytes_per_launch": round(sweep["bytes"] / max(1, sweep["launches"])),
            "launches": sweep["launches"],
            "avg_launch_us": round(sweep["ms"] * 1e3 / max(1, sweep["launches"]), 2)},
        "rounds": info["rounds"],
        "active_per_round": info["active"],
        "passes_per_round": info["passes_run"],
        "dense_rounds": info["dense_rounds"],
        "sigma": info["sigma"],
        "chars_round0": info["chars0"],
        "lazy_isa": info["lazy_isa"],
        "tuning": b.tuning(),
        "tuning_source": b.tuning_source(),
        "kernels": kernel_table(stats, steps),
        "wall_s": round(wall, 3),
    }
    log(f"{name}: {ms:.3f} ms/build, {value:.1f} Msuffixes/s, whole-build "
        f"{rec['whole_build_roofline']['frac']:.3f} of peak, sweep "
        f"{rec['sweep_roofline']['frac']:.3f}")
    if offsets is not None and per_text:
        # Per-text baseline on the same GPU: one sa_build per text, in order.
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for t in range(offsets.size - 1):
            a, z = int(offsets[t]), int(offsets[t + 1])
            if z > a:
                b.build(d_text[a:z], out=d_sa[a:z])
        e1.record(stream)
        torch.cuda.synchronize()
        per_text_ms = e0.elapsed_time(e1)
        pt_rate = n / (per_text_ms / 1e3) / 1e6
        rec["texts"] = int(offsets.size - 1)
        rec["per_text"] = {"msuffixes_s": round(pt_rate, 2), "ms": round(per_text_ms, 2)}
        rec["batched_vs_per_text"] = round(value / pt_rate, 3)
        log(f"{name}: per-text {pt_rate:.1f} Msuffixes/s -> batched x{value / pt_rate:.2f}")
    b.close()
    del d_text, d_sa
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rec["cpu_baseline"] = cpu_rows(name, text, offsets) if cpu else None
    return rec


# ---------------------------------------------------------------------------
# Rows beyond the headline path: prefix quadrupling, DC3, DC7, sort-based
# discarding and the index structures built from a suffix array. Each is
# checked against the headline path's suffix array of the same text and timed
# with HIP events; its kernel table comes from as many traced runs.

def _timed(fn, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _traced(b, fn, steps: int) -> dict:
    import torch
    b.reset_stats()
    b.set_trace(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    b.set_trace(False)
    return kernel_table(b.kernel_stats(), steps)


def _summary(name: str, n: int, ms: float, table: dict, extra: dict) -> dict:
    alg = sum(v["gb_s"] * v["ms_per_step"] / 1e3 for v in table.values())  # GB per step
    rec = {"workload": name, "n": n, "ms_per_build": round(ms, 4),
           "msuffixes_s": round(n / (ms / 1e3) / 1e6, 2),
           "whole_build_roofline": {
               "bound": "hbm", "algorithmic_gb": round(alg, 3),
               "achieved": round(alg / (ms / 1e3), 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(alg / (ms / 1e3) / HBM_PEAK_GBS, 4)},
           "kernels": table}
    rec.update(extra)
    log(f"{name}: {ms:.3f} ms, {rec['msuffixes_s']} Msuffixes/s, whole "
        f"{rec['whole_build_roofline']['frac']:.3f} of peak")
    return rec


def run_extras(steps: int = 2, warmup: int = 1) -> dict:
    import numpy as np
    import torch

    from paper_1610_03007_amd import SuffixArrayBuilder
    dev = torch.device("cuda", 0)
    out = {}
    b = SuffixArrayBuilder(0)

    # Prefix quadrupling on the repetitive 2^30 text (the most rounds).
    text, _ = make_text("repetitive_1g")
    n = int(text.size)
    d_text = torch.from_numpy(text).to(dev)
    ref = b.build(d_text)
    dbl = b.last_info()
    b.set_tuning(prefix_mult=4)
    sa = torch.empty_like(ref)
    ms = _timed(lambda: b.build(d_text, out=sa), steps, warmup)
    info = b.last_info()
    same = bool(torch.equal(sa, ref))
    table = _traced(b, lambda: b.build(d_text, out=sa), steps)
    b.auto_tuning()
    out["repetitive_1g_quadrupling"] = _summary(
        "repetitive_1g_quadrupling", n, ms, table,
        {"rounds": info["rounds"], "rounds_doubling": dbl["rounds"],
         "active_per_round": info["active"], "passes_per_round": info["passes_run"],
         "equals_doubling_sa": same})
    # DC7 on the same text: its work does not grow with the common prefixes.
    ms = _timed(lambda: b.build_dc7(d_text, out=sa), steps, warmup)
    info = b.last_info()
    same = bool(torch.equal(sa, ref))
    table = _traced(b, lambda: b.build_dc7(d_text, out=sa), 1)
    out["repetitive_1g_dc7"] = _summary(
        "repetitive_1g_dc7", n, ms, table,
        {"levels": info["rounds"], "level_sizes": info["active"], "equals_doubling_sa": same})
    del d_text, ref, sa
    torch.cuda.empty_cache()

    # DC3, DC7, sort-based discarding and the index structures on the Markov
    # 2^28 text.
    text, _ = make_text("markov_256m")
    n = int(text.size)
    d_text = torch.from_numpy(text).to(dev)
    ref = b.build(d_text)
    torch.cuda.synchronize()
    sa = torch.empty_like(ref)
    ms = _timed(lambda: b.build_dc3(d_text, out=sa), steps, warmup)
    info = b.last_info()
    same = bool(torch.equal(sa, ref))
    table = _traced(b, lambda: b.build_dc3(d_text, out=sa), 1)
    out["markov_256m_dc3"] = _summary(
        "markov_256m_dc3", n, ms, table,
        {"levels": info["rounds"], "level_sizes": info["active"], "equals_doubling_sa": same})
    ms = _timed(lambda: b.build_dc7(d_text, out=sa), steps, warmup)
    info = b.last_info()
    same = bool(torch.equal(sa, ref))
    table = _traced(b, lambda: b.build_dc7(d_text, out=sa), 1)
    out["markov_256m_dc7"] = _summary(
        "markov_256m_dc7", n, ms, table,
        {"levels": info["rounds"], "level_sizes": info["active"], "equals_doubling_sa": same})
    counts = [None]

    def sp():
        _, counts[0] = b.build_sorted_pairs(d_text, out=sa)
    ms = _timed(sp, steps, warmup)
    info = b.last_info()
    same = bool(torch.equal(sa, ref))
    table = _traced(b, sp, steps)
    out["markov_256m_sorted_pairs"] = _summary(
        "markov_256m_sorted_pairs", n, ms, table,
        {"rounds": info["rounds"], "counts_p_i_discarded_kept": counts[0].astype(int).tolist(),
         "equals_doubling_sa": same})

    # Index structures from the suffix array: bytes per suffix as counted by
    # the kernels (LCP 28, BWT 10, FM occurrence samples 1 + 8 sigma / 256).
    lcp = torch.empty_like(ref)
    ms_lcp = _timed(lambda: b.lcp(d_text, ref, out=lcp), steps, warmup)
    ms_bwt = _timed(lambda: b.bwt(d_text, ref), steps, warmup)
    fm = [None]

    def fm_build():
        if fm[0] is not None:
            fm[0].close()
        fm[0] = b.fm_index(d_text, ref)
    ms_fm = _timed(fm_build, steps, warmup)
    rng = np.random.default_rng(8)
    starts = rng.integers(0, n - 64, 1 << 16)
    pats = [text[s:s + int(rng.integers(4, 33))].tobytes() for s in starts]
    ranges = fm[0].count(pats)
    torch.cuda.synchronize()
    ms_q = _timed(lambda: fm[0].count(pats), steps, warmup)
    sigma = fm[0].info()["sigma"]
    fm[0].close()
    # Parity at full size on sampled rows: LCP by direct comparison, pattern
    # ranges contain the pattern's own start position.
    lc = lcp.cpu().numpy().view(np.uint32)
    sh = ref.cpu().numpy().view(np.uint32)
    rows = rng.integers(1, n, 2000)

    def lcp_direct(a: int, c: int, cap: int = 1 << 14) -> int:
        x, y = text[a:a + cap], text[c:c + cap]
        m = min(x.size, y.size)
        neq = np.nonzero(x[:m] != y[:m])[0]
        return int(neq[0]) if neq.size else (m if m < cap else -1)  # -1: at least cap

    lcp_ok = True
    for j in rows:
        d = lcp_direct(int(sh[j - 1]), int(sh[j]))
        lcp_ok &= (int(lc[j]) >= (1 << 14)) if d < 0 else int(lc[j]) == d
    rg = ranges.cpu().numpy()
    isa_pos = np.empty(n, dtype=np.int64)
    isa_pos[sh] = np.arange(n)
    q_ok = bool(all(rg[k, 0] <= isa_pos[starts[k]] < rg[k, 1] for k in range(0, len(pats), 64)))
    idx = {
        "lcp": {"ms": round(ms_lcp, 4), "gb_s": round(28.0 * n / ms_lcp / 1e6, 1)},
        "bwt": {"ms": round(ms_bwt, 4), "gb_s": round(10.0 * n / ms_bwt / 1e6, 1)},
        "fm_build": {"ms": round(ms_fm, 4),
                     "gb_s": round((1.0 + 8.0 * sigma / 256) * n / ms_fm / 1e6, 1)},
        "fm_count": {"patterns": len(pats), "ms": round(ms_q, 4),
                     "mpatterns_s": round(len(pats) / ms_q / 1e3, 2)},
        "lcp_sampled_rows_match": lcp_ok,
        "pattern_ranges_hold_their_start": q_ok,
    }
    for k in ("lcp", "bwt", "fm_build"):
        idx[k]["frac"] = round(idx[k]["gb_s"] / HBM_PEAK_GBS, 4)
    log(f"index: {idx}")
    out["markov_256m_index"] = idx
    b.close()
    del d_text, ref, sa, lcp
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# Serving.

def serve_stream(seconds: float, seed: int = 6):
    """Arrival times, lengths and generators of a Poisson request stream."""
    import numpy as np
    rng = np.random.default_rng(seed)
    count = int(SERVE_RATE * seconds * 1.2) + 16
    gaps = rng.exponential(1.0 / SERVE_RATE, count)
    t = np.cumsum(gaps)
    keep = t < seconds
    t = t[keep]
    n = np.floor(np.exp(rng.uniform(np.log(SERVE_LO), np.log(SERVE_HI), count)))[keep]
    kind = rng.integers(0, 2, count)[keep]
    off = rng.random(count)[keep]
    return t, n.astype(np.int64), kind, off


def serve_pools():
    """1 GiB of each source; requests are slices at random offsets (the sources
    are stationary, so a slice stands for a fresh draw)."""
    import workloads as W
    return [W.dna_long(1 << 30, seed=600), W.markov3(1 << 30, chain_seed=601)]


def run_server_load(pools, stream, warm: float, mode: str, digests: dict | None = None):
    """Replays the stream in real time. mode 'server': the continuous-batching
    server; 'per_text': one sa_build per request, first come first served.
    Returns (latencies of requests arriving after `warm` in ms, suffixes done in
    the window, window seconds, server stats). With `digests`, the SA of every
    16th request is hashed into it (key: request index) or compared with it."""
    import queue
    import threading

    import numpy as np
    import torch
    t_arr, lens, kind, off = stream
    texts = []
    for n, k, o in zip(lens, kind, off):
        pool = pools[int(k)]
        a = int(o * (pool.size - n))
        texts.append(pool[a:a + int(n)])
    lat = {}
    done_sufs = [0]
    mismatches = [0]

    def digest(i, sa_host):
        if digests is None or i % 16:
            return
        h = hashlib.sha256(np.ascontiguousarray(sa_host).view(np.uint8)).hexdigest()
        if i in digests:
            mismatches[0] += digests[i] != h
        else:
            digests[i] = h

    start = time.perf_counter() + 0.05
    if mode == "server":
        from paper_1610_03007_amd import SuffixArrayServer
        srv = SuffixArrayServer(0, capacity_bytes=96 << 30, max_text=SERVE_HI)
        tickets = {}
        lock = threading.Lock()
        finished = threading.Event()

        def producer():
            for i, ta in enumerate(t_arr):
                d = start + float(ta) - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tk = srv.submit(texts[i])
                with lock:
                    tickets[tk] = i
            finished.set()

        th = threading.Thread(target=producer)
        th.start()
        while True:
            with lock:
                pending = list(tickets.items())
            for tk, i in pending:
                ok, sa, ms = srv.poll(tk)
                if ok:
                    with lock:
                        del tickets[tk]
                    lat[i] = ms
                    digest(i, sa)
                    if t_arr[i] >= warm:
                        done_sufs[0] += int(lens[i])
            if finished.is_set() and not pending:
                with lock:
                    if not tickets:
                        break
            time.sleep(0.0005)
        th.join()
        stats = srv.stats()
        srv.close()
    else:
        from paper_1610_03007_amd import SuffixArrayBuilder
        b = SuffixArrayBuilder(0)
        dev = torch.device("cuda", 0)
        q = queue.Queue()

        def producer():
            for i, ta in enumerate(t_arr):
                d = start + float(ta) - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                q.put((i, time.perf_counter()))
            q.put(None)

        th = threading.Thread(target=producer)
        th.start()
        while True:
            item = q.get()
            if item is None:
                break
            i, t_sub = item
            d = torch.from_numpy(texts[i]).to(dev)
            sa = b.build(d)
            torch.cuda.synchronize()
            # Latency to the array ready on the device, as the server reports;
            # the caller then gets it in host memory, as from poll().
            lat[i] = (time.perf_counter() - t_sub) * 1e3
            host = torch.empty(sa.numel(), dtype=torch.int32, pin_memory=True)
            host.copy_(sa)
            digest(i, host.numpy())
            del sa, host
            if t_arr[i] >= warm:
                done_sufs[0] += int(lens[i])
        th.join()
        stats = None
        b.close()
    window = max(1e-9, (time.perf_counter() - start) - warm)
    ls = np.array([lat[i] for i in range(len(t_arr)) if t_arr[i] >= warm])
    return ls, done_sufs[0], window, stats, mismatches[0]


def run_serve(seconds: float, legs=("server", "per_text")) -> dict:
    import numpy as np
    t0 = time.perf_counter()
    pools = serve_pools()
    stream = serve_stream(seconds)
    log(f"serve: {len(stream[0])} requests over {seconds}s, {stream[1].sum() / 1e9:.2f} GB "
        f"of text; pools in {time.perf_counter() - t0:.1f}s")
    warm = min(2.0, seconds / 4)
    res = {}
    digests: dict = {}
    for mode in legs:
        ls, sufs, window, stats, bad = run_server_load(pools, stream, warm, mode, digests)
        res[mode] = {
            "requests": int(ls.size),
            "msuffixes_s": round(sufs / window / 1e6, 2),
            "p50_ms": round(float(np.percentile(ls, 50)), 3) if ls.size else None,
            "p99_ms": round(float(np.percentile(ls, 99)), 3) if ls.size else None,
            "mean_ms": round(float(ls.mean()), 3) if ls.size else None,
        }
        if stats:
            res[mode]["rounds"] = int(stats["rounds"])
            res[mode]["busy_ms"] = round(float(stats["busy_ms"]), 1)
        if mode == "per_text":
            res["served_equals_per_text"] = {"compared": len(digests), "mismatches": int(bad)}
        log(f"serve {mode}: {res[mode]}")
    # Capacity: the first requests of the stream all submitted at once.
    cap_n = int(np.searchsorted(stream[0], min(3.0, seconds)))
    sat = (np.zeros(cap_n), stream[1][:cap_n], stream[2][:cap_n], stream[3][:cap_n])
    for mode in legs:
        ls, sufs, window, _, _ = run_server_load(pools, sat, 0.0, mode)
        res[mode]["capacity_msuffixes_s"] = round(sufs / window / 1e6, 2)
        res[mode]["capacity_requests"] = cap_n
        log(f"serve {mode} capacity: {res[mode]['capacity_msuffixes_s']} Msuffixes/s")
    offered = float(stream[1][stream[0] >= warm].sum()) / (seconds - warm) / 1e6
    if tuple(legs) != ("server", "per_text"):
        return {"workload": "serve", "seconds": seconds, "warmup_s": warm,
                "offered_msuffixes_s": round(offered, 2), "legs": list(legs), **res}
    return {
        "workload": "serve",
        "description": WORKLOADS["serve"],
        "seconds": seconds,
        "warmup_s": warm,
        "offered_msuffixes_s": round(offered, 2),
        "msuffixes_s": res["server"]["msuffixes_s"],
        "p50_ms": res["server"]["p50_ms"],
        "p99_ms": res["server"]["p99_ms"],
        "server": res["server"],
        "per_text": res["per_text"],
        "served_equals_per_text": res["served_equals_per_text"],
        "p99_per_text_over_server": (round(res["per_text"]["p99_ms"] / res["server"]["p99_ms"], 3)
                                     if res["server"]["p99_ms"] else None),
        "capacity_server_over_per_text": round(
            res["server"]["capacity_msuffixes_s"] / res["per_text"]["capacity_msuffixes_s"], 3),
    }


# ---------------------------------------------------------------------------

def headline(rec: dict, steps: int, warmup: int, workload: str) -> dict:
    """The driver's JSON line for a build record."""
    sweep = rec["sweep_roofline"]
    config = {"workload": workload, "description": rec["description"], "n": rec["n"],
              "rounds": rec["rounds"], "active_per_round": rec["active_per_round"],
              "parallelism": "single GPU", "tuning": rec["tuning"],
              "tuning_source": rec["tuning_source"]}
    if "texts" in rec:
        config["texts"] = rec["texts"]
    return {
        "metric": METRIC,
        "value": rec["msuffixes_s"],
        "unit": "Msuffixes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": rec["ms_per_build"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": config,
        "roofline": {k: sweep[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                          "traffic")} | {
            "kernel": sweep["kernel"], "launches": sweep["launches"],
            "avg_launch_us": sweep["avg_launch_us"],
            "algorithmic_bytes_per_launch": sweep["algorithmic_bytes_per_launch"]},
        "whole_build_roofline": rec["whole_build_roofline"],
        "cpu_baseline": rec["cpu_baseline"],
    }


def tune_main(args) -> int:
    """Autotunes each listed workload (one text, or the batch) and writes the
    cache table; one progress line per workload."""
    import torch

    from paper_1610_03007_amd import SuffixArrayBuilder
    os.environ.setdefault("SA_TUNE_LOG", "1")  # one line per candidate: progress on stderr
    dev = torch.device("cuda", 0)
    b = SuffixArrayBuilder(0, tune_cache=args.tune)
    for name in [w for w in args.tune_workloads.split(",") if w]:
        t0 = time.perf_counter()
        text, offsets = make_text(name)
        d_text = torch.from_numpy(text).to(dev)
        best, ms = b.tune(d_text, offsets, reps=args.tune_reps)
        b.save_tuning()
        print(json.dumps({"tune": name, "n": int(text.size), "best": best, "ms": round(ms, 3),
                          "msuffixes_s": round(text.size / ms / 1e3, 1),
                          "wall_s": round(time.perf_counter() - t0, 1)}), flush=True)
        del d_text
        torch.cuda.empty_cache()
    b.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all", choices=["all"] + sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle rows")
    ap.add_argument("--no-per-text", action="store_true",
                    help="batch workload: skip the one-sa_build-per-text baseline (profiling)")
    ap.add_argument("--serve-legs", default="server,per_text",
                    help="serve workload: which legs to run (server, per_text or both)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip quadrupling, DC3, DC7, sort-based discarding and the index rows")
    ap.add_argument("--extras-only", action="store_true",
                    help="run only those rows (one JSON object)")
    ap.add_argument("--sort-items", type=int, default=0,
                    help="radix-sort items per thread (0 = library default)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the replayed request stream (serve workload)")
    ap.add_argument("--tune", metavar="OUT_JSON", default="",
                    help="run the autotuner on --tune-workloads and write the cache table "
                         "to OUT_JSON instead of benchmarking")
    ap.add_argument("--tune-workloads", default="dna_1m,markov_256m,repetitive_1g,batch_4096")
    ap.add_argument("--tune-reps", type=int, default=2)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB of a plain device copy to run after the steps (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the texts of a batch would shard across GPUs without any exchange, but a "
              f"single text needs an all-to-all exchange per round, which is not built).",
              file=sys.stderr)
        return 2
    if args.tune:
        return tune_main(args)
    cpu = not args.no_cpu

    if args.extras_only:
        print(json.dumps(run_extras()), flush=True)
        return 0
    if args.workload == "serve":
        rec = run_serve(args.serve_seconds, tuple(x for x in args.serve_legs.split(",") if x))
        if "msuffixes_s" not in rec:
            rec["msuffixes_s"] = rec[rec["legs"][0]]["msuffixes_s"]
        out = {"metric": METRIC, "value": rec["msuffixes_s"], "unit": "Msuffixes/s",
               "n_gpus": 1, "steps": 1, "warmup": 0,
               "ms_per_step": round(args.serve_seconds * 1e3, 1), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
               "config": {"workload": "serve", "parallelism": "single GPU"},
               "roofline": None, "cpu_baseline": None, "serve": rec}
        print(json.dumps(out), flush=True)
        return 0

    names = BUILD_ORDER if args.workload == "all" else (args.workload,)
    records = {}
    for name in names:
        # The headline workload takes the driver's step counts; the others are
        # bounded so that the whole run stays within a few minutes.
        steps, warmup = args.steps, args.warmup
        if name != names[0]:
            if name == "repetitive_1g":
                steps, warmup = min(steps, 3), min(warmup, 1)
            elif name == "dna_1m":
                steps = max(steps, 20)
        records[name] = run_build(name, steps, warmup, cpu, args.sort_items,
                                  per_text=not args.no_per_text)
    head = names[0]
    out = headline(records[head], args.steps, args.warmup, head)
    if args.workload == "all":
        records["serve"] = run_serve(args.serve_seconds)
        if not args.no_extras:
            records.update(run_extras())
    out["configs"] = {k: v for k, v in records.items() if k != head}
    out["batch"] = ({"texts": records[head]["texts"],
                     "batched_msuffixes_s": records[head]["msuffixes_s"],
                     "per_text_msuffixes_s": records[head]["per_text"]["msuffixes_s"],
                     "batched_vs_per_text": records[head]["batched_vs_per_text"]}
                    if "per_text" in records[head] else None)
    if "serve" in records:
        s = records["serve"]
        out["serve"] = {"p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"],
                        "msuffixes_s": s["msuffixes_s"],
                        "capacity_server_over_per_text": s["capacity_server_over_per_text"]}
    out["kernels"] = records[head]["kernels"]

    if args.calibrate_copy > 0:
        import torch
        nbytes = args.calibrate_copy << 20
        dev = torch.device("cuda", 0)
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibrate_copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
