#!/usr/bin/env python3
"""Benchmark: suffix-array construction throughput on one MI355X.

One step = one complete sa_build (every doubling round: key packing, radix
sort, re-rank / ISA scatter / discard) of the 256 MiB order-3 Markov text over
96 printable bytes, with the text already resident in HBM. Prints one JSON line
with Msuffixes/s, the HBM roofline of the dominant kernel (the radix-sort
sweep) measured with HIP events inside the timed steps, and the CPU oracle
timed on a bounded sample on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
WORKLOADS = {
    "markov_256m": "order-3 Markov text, 96 printable bytes, Dirichlet(0.1) rows, n=2^28",
    "dna_1m": "uniform ACGT text, seed 0, n=2^20",
    "repetitive_1g": "256 KiB base x 4096 copies, 1e-4 substitutions, n=2^30",
    "batch_4096": "4096 texts, lengths log-uniform in [4 KiB, 8 MiB], half ACGT, half "
                  "order-3 Markov (96 bytes); one batched build",
    "serve": "Poisson arrivals at 330.5 req/s (2 GB/s of text), lengths log-uniform in "
             "[1 KiB, 64 MiB], ACGT or Markov slices; continuous-batching server",
}
SERVE_RATE = 330.5
SERVE_LO, SERVE_HI = 1024, 1 << 26
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_03007_amd", "csrc", "sa_kernels.hip")


def make_text(name: str):
    """Returns (text, offsets or None)."""
    import workloads as W
    if name == "batch_4096":
        return W.batch()
    return make_single(name), None


def make_single(name: str):
    import workloads as W
    if name == "markov_256m":
        return W.markov3(1 << 28, chain_seed=2)
    if name == "dna_1m":
        return W.dna(1 << 20, seed=0)
    if name == "repetitive_1g":
        return W.repetitive()
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def cpu_baseline(text, sample: int, offsets=None):
    import oracle
    if offsets is None:
        s = text[:sample].copy()
        t0 = time.perf_counter()
        oracle.sa(s, parallel=True)
        dt = time.perf_counter() - t0
        total = s.size
        what = f"first {s.size} bytes of the same text"
    else:
        # Whole texts of the batch, in order, until the sample size is reached.
        t0 = time.perf_counter()
        total = ntexts = 0
        for t in range(offsets.size - 1):
            a, b = int(offsets[t]), int(offsets[t + 1])
            oracle.sa(text[a:b], parallel=True)
            total += b - a
            ntexts += 1
            if total >= sample:
                break
        dt = time.perf_counter() - t0
        what = f"the first {ntexts} texts of the batch ({total} bytes), one oracle call per text"
    return {
        "value": round(total / dt / 1e6, 3),
        "unit": "Msuffixes/s",
        "cores": oracle.num_threads(parallel=True),
        "kind": "oracle",
        "sample": f"{what}, plain prefix doubling (GNU parallel std::sort), {dt:.2f} s",
    }


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
    return [W.dna(1 << 30, seed=600), W.markov3(1 << 30, chain_seed=601)]


def run_server_load(pools, stream, warm: float, mode: str):
    """Replays the stream in real time. mode 'server': the continuous-batching
    server; 'per_text': one sa_build per request, first come first served.
    Returns (latencies of requests arriving after `warm` in ms, suffixes done in
    the window, window seconds)."""
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
    t_end = float(t_arr[-1]) if len(t_arr) else 0.0
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
            del sa, host
            if t_arr[i] >= warm:
                done_sufs[0] += int(lens[i])
        th.join()
        stats = None
        b.close()
    window = max(1e-9, (time.perf_counter() - start) - warm)
    ls = np.array([lat[i] for i in range(len(t_arr)) if t_arr[i] >= warm])
    return ls, done_sufs[0], window, stats


def serve_main(args) -> int:
    import numpy as np
    t0 = time.perf_counter()
    pools = serve_pools()
    stream = serve_stream(args.serve_seconds)
    print(f"[bench] serve: {len(stream[0])} requests over {args.serve_seconds}s, "
          f"{stream[1].sum() / 1e9:.2f} GB of text; pools in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    warm = min(2.0, args.serve_seconds / 4)
    res = {}
    for mode in ("server", "per_text"):
        ls, sufs, window, stats = run_server_load(pools, stream, warm, mode)
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
        print(f"[bench] {mode}: {res[mode]}", file=sys.stderr, flush=True)
    # Capacity: the first requests of the stream all submitted at once.
    cap_n = int(np.searchsorted(stream[0], min(4.0, args.serve_seconds)))
    sat = (np.zeros(cap_n), stream[1][:cap_n], stream[2][:cap_n], stream[3][:cap_n])
    for mode in ("server", "per_text"):
        ls, sufs, window, _ = run_server_load(pools, sat, 0.0, mode)
        res[mode]["capacity_msuffixes_s"] = round(sufs / window / 1e6, 2)
        res[mode]["capacity_requests"] = cap_n
        print(f"[bench] {mode} capacity: {res[mode]['capacity_msuffixes_s']} Msuffixes/s",
              file=sys.stderr, flush=True)
    offered = float(stream[1][stream[0] >= warm].sum()) / (args.serve_seconds - warm) / 1e6
    result = {
        "metric": "Msuffixes/s on 1 GPU + HBM roofline %; batched vs per-text; p50/p99 latency",
        "value": res["server"]["msuffixes_s"],
        "unit": "Msuffixes/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(args.serve_seconds * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serve", "description": WORKLOADS["serve"],
                   "seconds": args.serve_seconds, "warmup_s": warm,
                   "offered_msuffixes_s": round(offered, 2), "parallelism": "single GPU"},
        "serve": {
            "p50_ms": res["server"]["p50_ms"], "p99_ms": res["server"]["p99_ms"],
            "server": res["server"], "per_text": res["per_text"],
            "p99_per_text_over_server": (round(res["per_text"]["p99_ms"] / res["server"]["p99_ms"], 3)
                                         if res["server"]["p99_ms"] else None),
            "capacity_server_over_per_text": round(
                res["server"]["capacity_msuffixes_s"] / res["per_text"]["capacity_msuffixes_s"], 3),
        },
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)
    return 0


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
    ap.add_argument("--workload", default="markov_256m", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=1 << 28,
                    help="bytes of the text the CPU oracle is timed on (0 = skip; batches "
                         "are sampled by whole texts)")
    ap.add_argument("--sort-items", type=int, default=0,
                    help="radix-sort items per thread (0 = library default)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
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
              f"(a single text does not shard without an all-to-all exchange step).",
              file=sys.stderr)
        return 2

    if args.workload == "serve":
        return serve_main(args)
    if args.tune:
        return tune_main(args)

    import numpy as np
    import torch

    from paper_1610_03007_amd import SuffixArrayBuilder

    t_gen = time.perf_counter()
    text, offsets = make_text(args.workload)
    n = int(text.size)
    print(f"[bench] workload {args.workload} n={n} generated in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    d_text = torch.from_numpy(text).to(dev)
    d_sa = torch.empty(n, dtype=torch.int32, device=dev)
    b = SuffixArrayBuilder(0)
    if args.sort_items:
        b.set_tuning(sort_items=args.sort_items)

    def step():
        if offsets is None:
            b.build(d_text, out=d_sa)
        else:
            b.build_batch(d_text, offsets, out=d_sa)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done: {b.last_info()}", file=sys.stderr, flush=True)

    b.reset_stats()
    b.set_trace(True)
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.set_trace(False)
    gpu_ms = ev0.elapsed_time(ev1)
    info = b.last_info()
    stats = b.kernel_stats()

    ms_per_step = gpu_ms / args.steps
    value = n * args.steps / (gpu_ms / 1e3) / 1e6

    sweep = stats["sort_pass"]
    achieved = sweep["bytes"] / (sweep["ms"] / 1e3) / 1e9 if sweep["ms"] > 0 else 0.0
    per_launch = sweep["bytes"] / max(1, sweep["launches"])
    traffic = measured_traffic(args.workload)

    result = {
        "metric": "Msuffixes/s on 1 GPU + HBM roofline %; batched vs per-text; p50/p99 latency",
        "value": round(value, 2),
        "unit": "Msuffixes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "description": WORKLOADS[args.workload],
            "n": n,
            "rounds": info["rounds"],
            "active_per_round": info["active"],
            "sigma": info["sigma"],
            "chars_round0": info["chars0"],
            "parallelism": "single GPU",
            "tuning": b.tuning(),
            "tuning_source": b.tuning_source(),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "onesweep_pass_kernel",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(per_launch),
            "launches": sweep["launches"],
            "avg_launch_us": round(sweep["ms"] * 1e3 / max(1, sweep["launches"]), 2),
        },
        "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in stats.items()},
        "wall_s": round(wall, 3),
    }
    if offsets is not None:
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
        per_text = n / (per_text_ms / 1e3) / 1e6
        result["batch"] = {
            "texts": int(offsets.size - 1),
            "batched_msuffixes_s": round(value, 2),
            "per_text_msuffixes_s": round(per_text, 2),
            "per_text_ms": round(per_text_ms, 2),
            "batched_vs_per_text": round(value / per_text, 3),
        }
    if args.cpu_sample > 0:
        result["cpu_baseline"] = cpu_baseline(text, min(args.cpu_sample, n), offsets)
    else:
        result["cpu_baseline"] = None

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["calibrate_copy_bytes"] = nbytes

    b.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
