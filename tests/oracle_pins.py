"""Compact pin set for the oracle, run in its own interpreter.

Usage: python oracle_pins.py [path/to/liboracle_variant.so]
Exits 0 when every pin holds for the given build of the oracle (default: the
normal build), 1 otherwise. Used to show that planted mistakes in the oracle
source are caught. Expected values come from the paper's examples, closed forms
and a brute-force sort written here in Python, never from the oracle.
"""

import ctypes
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def py_brute_sa(t: bytes):
    return sorted(range(len(t)), key=lambda i: t[i:])


def py_prefix_ranks(t: bytes, h: int):
    pads = [t[i:i + h] for i in range(len(t))]
    first = {}
    for pos, p in enumerate(sorted(pads)):
        first.setdefault(p, pos)
    return [first[p] + 1 for p in pads]


def py_lcp(t: bytes):
    sa = py_brute_sa(t)
    out = [0] * len(t)
    for j in range(1, len(t)):
        a, b = t[sa[j - 1]:], t[sa[j]:]
        l = 0
        while l < min(len(a), len(b)) and a[l] == b[l]:
            l += 1
        out[j] = l
    return out


def py_bwt(t: bytes):
    """Last column of the sorted rotations of t$ ($ = -1, below every byte)."""
    seq = list(t) + [-1]
    m = len(seq)
    rows = sorted(range(m), key=lambda i: seq[i:] + seq[:i])
    col = [seq[(i - 1) % m] for i in rows]
    d = col.index(-1)
    return bytes(c for c in col if c >= 0), d


def py_interval(t: bytes, p: bytes):
    sa = py_brute_sa(t)
    m = len(p)
    lo = sum(1 for s in sa if t[s:s + m] < p)
    occ = sum(1 for i in range(len(t)) if t[i:i + m] == p)
    return lo, lo + occ


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def pdd_pins(rng) -> bool:
    """Sort-based prefix doubling with discarding (Alg. 5)."""
    g = load("paper_example1_comparator.json")
    t = g["text"].encode()
    for h, printed in g["comparator_sorted_printed"].items():
        if oracle.opk_order(len(t), int(h)).tolist() != [p[0] for p in printed]:
            return False
    # With c = 2 (the paper's initial pairs) the working items of rounds 1 and
    # 2 are the printed lists: every non-unique item is in them, and the one
    # unique item (position 8) is kept while two non-unique items precede it.
    for k, h in ((1, "2"), (2, "4")):
        pos, names, uniq = oracle.pdd_round(t, 2, k)
        printed = g["comparator_sorted_printed"][h]
        if pos.tolist() != [p[0] for p in printed] or \
                names.tolist() != [p[1] + 1 for p in printed]:
            return False
    pos, names, _ = oracle.pdd_round(t, 2, 1)
    pairs = [(int(pos[p]), int(names[p]),
              int(names[p + 1]) if p + 1 < len(pos) and pos[p + 1] == pos[p] + 2 else 0)
             for p in range(len(pos))]
    # Printed names are 0-based; the partner's name is the sentinel when
    # suffix i + 2 does not exist.
    want = [(i, a + 1, b + 1 if i + 2 < len(t) else 0) for i, a, b in g["pairs_printed"]["2"]]
    if pairs != want:
        return False
    g = load("pdd_worked_aba.json")
    sa, counts = oracle.pdd_sa(g["text"].encode(), g["c"])
    if sa.tolist() != g["sa"] or counts.astype(int).tolist() != g["counts"]:
        return False
    for _ in range(40):
        n = int(rng.integers(1, 100))
        tt = rng.integers(0, int(rng.choice([1, 2, 3, 256])), n).astype(np.uint8)
        tb = tt.tobytes()
        c = int(rng.choice([1, 2, 3, 8]))
        sa, counts = oracle.pdd_sa(tt, c)
        if sa.tolist() != py_brute_sa(tb):
            return False
        P, I, D, U = (counts[:, j].astype(int).tolist() for j in range(4))
        if P[0] != n or sum(D) != n or I[-1] != 0 or U[-1] != 0:
            return False
        for k in range(len(P)):
            if P[k] != I[k] + D[k] + U[k]:
                return False
            if k + 1 < len(P) and P[k + 1] != I[k] + U[k]:
                return False
            h = c << k
            got = oracle.pdd_round(tt, c, k + 1)
            if got is None:
                return False
            pos, names, uniq = got
            # Names are the closed form at prefix length h, unique flags agree
            # with them, and every non-unique item finds suffix i + h present.
            want = py_prefix_ranks(tb, h)
            if names.tolist() != [want[i] for i in pos.tolist()]:
                return False
            present = set(pos.tolist())
            for i, u in zip(pos.tolist(), uniq.tolist()):
                if u != (want.count(want[i]) == 1):
                    return False
                if not u and i + h < n and i + h not in present:
                    return False
    return True


def pins_pass() -> bool:
    for fixture in ("paper_example1_bdacbdacb.json", "banana.json"):
        g = load(fixture)
        t = g["text"].encode()
        if oracle.sa(t).tolist() != g["sa"] or oracle.brute_sa(t).tolist() != g["sa"]:
            return False
    g = load("paper_example1_bdacbdacb.json")
    t = g["text"].encode()
    for steps, h in ((1, 2), (2, 4)):
        names, h_got = oracle.pd_names(t, steps)
        if h_got != h or names.tolist() != py_prefix_ranks(t, h):
            return False
        if oracle.prefix_ranks(t, h).tolist() != py_prefix_ranks(t, h):
            return False
    if oracle.sa(b"a\0\0").tolist() != [2, 1, 0]:
        return False
    m = 9
    if oracle.sa(b"ab" * m).tolist() != list(range(2 * m - 2, -1, -2)) + list(range(2 * m - 1, 0, -2)):
        return False
    rng = np.random.default_rng(11)
    for _ in range(60):
        n = int(rng.integers(2, 120))
        t = rng.integers(0, int(rng.choice([2, 4, 256])), n).astype(np.uint8)
        want = py_brute_sa(t.tobytes())
        if oracle.sa(t).tolist() != want or oracle.brute_sa(t).tolist() != want:
            return False
        if oracle.prefix_ranks(t, 3).tolist() != py_prefix_ranks(t.tobytes(), 3):
            return False
        names, h = oracle.pd_names(t, 2)
        if names.tolist() != py_prefix_ranks(t.tobytes(), h):
            return False
        bad = np.array(want, dtype=np.uint32)
        j = int(rng.integers(0, n - 1))
        bad[j], bad[j + 1] = bad[j + 1], bad[j]
        if oracle.check_sa(t, bad)[0] != 2:
            return False
        tb = t.tobytes()
        sa = np.array(want, dtype=np.uint32)
        if oracle.lcp(t, sa).tolist() != py_lcp(tb):
            return False
        bw, d = oracle.bwt(t, sa)
        if (bw.tobytes(), d) != py_bwt(tb):
            return False
        for _ in range(3):
            a = int(rng.integers(0, n))
            pat = tb[a:a + int(rng.integers(0, 4))] if rng.random() < 0.7 else \
                bytes(rng.integers(0, 3, int(rng.integers(1, 4))).astype(np.uint8))
            if oracle.sa_interval(t, sa, pat) != py_interval(tb, pat):
                return False
    # Prefix a-tupling: after k sorts the names resolve prefix length a^k.
    for a in (2, 3, 4):
        for _ in range(12):
            n = int(rng.integers(2, 90))
            t = rng.integers(0, int(rng.choice([2, 3, 256])), n).astype(np.uint8)
            tb = t.tobytes()
            if oracle.pa_sa(t, a).tolist() != py_brute_sa(tb):
                return False
            for k in range(0, 4):
                names, h = oracle.pa_names(t, a, k)
                if h > a ** k or names.tolist() != py_prefix_ranks(tb, h):
                    return False
                if h == a ** k and k > 0 and len(set(py_prefix_ranks(tb, a ** (k - 1)))) == n:
                    return False  # names were distinct already: no further sort runs
    if oracle.pa_sa(b"aaaaaaaaaaaaaaaaaaaaaaaa", 4).tolist() != list(range(23, -1, -1)):
        return False
    if not pdd_pins(rng):
        return False
    g = load("paper_example3_dbacbacbd.json")
    r1, r2 = oracle.dc3_sample_ranks(g["text"].encode())
    if r1.tolist() != g["dc3_r1"] or r2.tolist() != g["dc3_r2"]:
        return False
    for _ in range(30):
        n = int(rng.integers(1, 80))
        tt = rng.integers(0, int(rng.choice([1, 2, 3, 256])), n).astype(np.uint8)
        sample = [i for i in py_brute_sa(tt.tobytes()) if i % 3]
        rank = {i: k + 1 for k, i in enumerate(sample)}
        r1, r2 = oracle.dc3_sample_ranks(tt)
        if r1.tolist() != [rank[i] for i in range(1, n, 3)] or \
                r2.tolist() != [rank[i] for i in range(2, n, 3)]:
            return False
        # DC7's cover {0, 1, 3} mod 7 (and DC3's, through the general form).
        for x, cover in ((7, (0, 1, 3)), (3, (1, 2))):
            sample = [i for i in py_brute_sa(tt.tobytes()) if i % x in cover]
            want = [0] * n
            for k, i in enumerate(sample):
                want[i] = k + 1
            if oracle.dcx_sample_ranks(tt, x, cover).tolist() != want:
                return False
    if oracle.lcp(b"banana", [5, 3, 1, 0, 4, 2]).tolist() != [0, 1, 3, 0, 0, 2]:
        return False
    bw, d = oracle.bwt(b"banana", [5, 3, 1, 0, 4, 2])
    if (bw.tobytes(), d) != (b"annbaa", 4):
        return False
    return True


if __name__ == "__main__":
    if len(sys.argv) > 1:
        oracle._libs[False] = oracle.configure(ctypes.CDLL(sys.argv[1]))
    try:
        ok = pins_pass()
    except Exception:
        ok = False
    sys.exit(0 if ok else 1)
