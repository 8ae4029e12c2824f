"""Pins for the CPU oracle (no GPU).

Every expected value here comes from outside the oracle: the paper's worked
examples (fixtures under tests/golden, each with its citation), a brute-force
suffix sort written independently in Python, closed forms for structured texts,
and planted mistakes (mutants of the oracle source) that these pins must catch.
"""

import itertools
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PINS = os.path.join(os.path.dirname(__file__), "oracle_pins.py")


def py_brute_sa(t: bytes):
    """Definition of the suffix array: Python bytes compare as unsigned bytes and
    a proper prefix is smaller than its extensions."""
    return [i for i in sorted(range(len(t)), key=lambda i: t[i:])]


def py_prefix_ranks(t: bytes, h: int):
    """Closed form: 1 + number of positions whose padded length-h prefix is smaller."""
    pads = [t[i:i + h] for i in range(len(t))]
    order = sorted(pads)
    first = {}
    for pos, p in enumerate(order):
        first.setdefault(p, pos)
    return [first[p] + 1 for p in pads]


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Paper worked examples and the textbook example.

@pytest.mark.parametrize("fixture", ["paper_example1_bdacbdacb.json",
                                     "paper_example3_dbacbacbd.json", "banana.json"])
def test_golden_sa(fixture):
    g = load(fixture)
    t = g["text"].encode()
    assert oracle.sa(t).tolist() == g["sa"]
    assert oracle.brute_sa(t).tolist() == g["sa"]
    assert oracle.check_sa(t, g["sa"]) == (0, 0)


def test_golden_round_names():
    """Names printed after each doubling iteration (Examples 1 and 2) equal both
    the oracle's doubling names and its closed form, shifted to 1-based."""
    g = load("paper_example1_bdacbdacb.json")
    t = g["text"].encode()
    for step, (h, tuples) in enumerate(sorted(g["names_printed"].items(),
                                              key=lambda kv: int(kv[0])), start=1):
        h = int(h)
        want = np.zeros(len(t), dtype=np.uint32)
        for pos, name in tuples:
            want[pos] = name + 1
        names, h_got = oracle.pd_names(t, step)
        assert h_got == h
        assert names.tolist() == want.tolist()
        assert oracle.prefix_ranks(t, h).tolist() == want.tolist()


# --------------------------------------------------------------------------
# Brute force on small inputs.

def test_all_binary_strings():
    for n in range(0, 13):
        for bits in itertools.product(b"ab", repeat=n):
            t = bytes(bits)
            want = py_brute_sa(t)
            assert oracle.sa(t).tolist() == want, t
    # spot-check length 14 (exhaustive 2^14 also passes but costs time)
    rng = np.random.default_rng(7)
    for _ in range(500):
        t = bytes(rng.choice([97, 98], 14).astype(np.uint8))
        assert oracle.sa(t).tolist() == py_brute_sa(t)


@pytest.mark.parametrize("sigma", [1, 2, 4, 96, 256])
def test_random_strings(sigma):
    rng = np.random.default_rng(100 + sigma)
    for _ in range(300):
        n = int(rng.integers(0, 400))
        t = rng.integers(0, sigma, n).astype(np.uint8)
        if sigma == 96:
            t = np.where(t == 0, 10, t + 31).astype(np.uint8)
        tb = t.tobytes()
        want = py_brute_sa(tb)
        assert oracle.sa(t).tolist() == want
        assert oracle.brute_sa(t).tolist() == want
        assert oracle.check_sa(t, want) == (0, 0)


def test_prefix_ranks_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(1, 200))
        sigma = int(rng.choice([1, 2, 3, 256]))
        t = rng.integers(0, sigma, n).astype(np.uint8).tobytes()
        h = int(rng.integers(1, 40))
        assert oracle.prefix_ranks(t, h).tolist() == py_prefix_ranks(t, h)


def test_doubling_names_match_closed_form():
    rng = np.random.default_rng(4)
    for _ in range(100):
        n = int(rng.integers(2, 300))
        t = rng.integers(0, 3, n).astype(np.uint8).tobytes()
        for steps in (1, 2, 3, 4):
            names, h = oracle.pd_names(t, steps)
            assert names.tolist() == py_prefix_ranks(t, h)


# --------------------------------------------------------------------------
# Closed forms and special cases.

def test_edge_sizes():
    assert oracle.sa(b"").tolist() == []
    assert oracle.sa(b"x").tolist() == [0]
    assert oracle.sa(b"ab").tolist() == [0, 1]
    assert oracle.sa(b"ba").tolist() == [1, 0]
    assert oracle.sa(b"aa").tolist() == [1, 0]


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 4097])
def test_unary(n):
    assert oracle.sa(b"a" * n).tolist() == list(range(n - 1, -1, -1))


def test_monotone():
    inc = bytes(range(256))
    assert oracle.sa(inc).tolist() == list(range(256))
    dec = bytes(range(255, -1, -1))
    assert oracle.sa(dec).tolist() == list(range(255, -1, -1))


@pytest.mark.parametrize("m", [1, 2, 5, 64, 333])
def test_ab_repeats(m):
    # (ab)^m: the a-suffixes in order of increasing length, then the b-suffixes.
    want = list(range(2 * m - 2, -1, -2)) + list(range(2 * m - 1, 0, -2))
    assert oracle.sa(b"ab" * m).tolist() == want


def test_nul_bytes():
    assert oracle.sa(b"a\0\0").tolist() == [2, 1, 0]
    assert oracle.sa(b"\0\0\0\0").tolist() == [3, 2, 1, 0]
    t = b"\0a\0a\0"
    assert oracle.sa(t).tolist() == py_brute_sa(t)


# --------------------------------------------------------------------------
# Checker.

def test_checker_rejects():
    rng = np.random.default_rng(9)
    for _ in range(300):
        n = int(rng.integers(2, 200))
        t = rng.integers(0, int(rng.choice([2, 4, 256])), n).astype(np.uint8)
        good = np.array(py_brute_sa(t.tobytes()), dtype=np.uint32)
        assert oracle.check_sa(t, good) == (0, 0)
        bad = good.copy()
        j = int(rng.integers(0, n - 1))
        bad[j], bad[j + 1] = bad[j + 1], bad[j]
        assert oracle.check_sa(t, bad)[0] == 2
        dup = good.copy()
        dup[j] = dup[j + 1]
        assert oracle.check_sa(t, dup)[0] == 1
        rng_perm = rng.permutation(n).astype(np.uint32)
        if not np.array_equal(rng_perm, good):
            assert oracle.check_sa(t, rng_perm)[0] == 2


# --------------------------------------------------------------------------
# Planted mistakes: each mutant of the oracle source must fail some pin above.

MUTANTS = {
    "sentinel_largest": ("uint64_t r1 = (i + h < n) ? name[i + h] : 0;",
                         "uint64_t r1 = (i + h < n) ? name[i + h] : 0xFFFFFFFFull;"),
    "unshifted_next": ("? uint64_t(T[i + 1]) + 1 : 0;", "? uint64_t(T[i + 1]) : 0;"),
    "zero_based_names": ("name[S[p].i] = static_cast<uint32_t>(last_head + 1);",
                         "name[S[p].i] = static_cast<uint32_t>(last_head);"),
    "offset_off_by_one": ("(i + h < n) ? name[i + h] : 0;", "(i + h < n) ? name[i + h - 1] : 0;"),
    "dropped_second_rank": ("S[i] = Triple{(r0 << 32) | r1, static_cast<uint32_t>(i)};",
                            "S[i] = Triple{(r0 << 32), static_cast<uint32_t>(i)};"),
    "early_stop": ("if (distinct == n) break;", "if (distinct + 1 >= n) break;"),
    "no_doubling": ("    h *= 2;\n  }\n  if (h_out) *h_out = h;", "    h += 1;\n  }\n  if (h_out) *h_out = h;"),
    "pdd_no_doubling": ("    h *= 2;\n  }\n  return round;", "    h += 1;\n  }\n  return round;"),
    "prefix_longer_first": ("return li < lj ? -1 : 1;", "return li < lj ? 1 : -1;"),
    "checker_loose": ("bool ok = (T[a] < T[b]) ||", "bool ok = (T[a] <= T[b]) ||"),
    "lcp_overcount": ("lcp[j] = static_cast<uint32_t>(l);",
                      "lcp[j] = static_cast<uint32_t>(l + (l > 0));"),
    "bwt_unshifted": ("out[k++] = T[SA[j] - 1];", "out[k++] = T[SA[j]];"),
    "bwt_dollar_row": ("*dollar = j + 1;", "*dollar = j;"),
    "interval_open_end": ("if (cmp_prefix(T, n, SA[mid], P, m) <= 0)",
                          "if (cmp_prefix(T, n, SA[mid], P, m) < 0)"),
    "interval_short_suffix_larger": ("if (s + l >= n) return -1;", "if (s + l >= n) return 1;"),
    "tuple_last_rank_dropped": ("for (uint32_t j = 0; j < a; ++j) {",
                                "for (uint32_t j = 0; j + 1 < a; ++j) {"),
    "tuple_offset_stride": ("const uint64_t q = i + uint64_t(j) * h;",
                            "const uint64_t q = i + uint64_t(j) * (h > 1 ? h / 2 : 1);"),
    "tuple_h_doubled": ("    h *= a;\n    ++done;", "    h *= 2;\n    ++done;"),
    "tuple_char_names_zero": ("name[i] = static_cast<uint32_t>(below[T[i]] + 1);",
                              "name[i] = static_cast<uint32_t>(below[T[i]]);"),
    "pdd_keep_after_one": ("} else if (p >= 2 && P[p - 1].s == 'n' && P[p - 2].s == 'n') {",
                           "} else if (p >= 1 && P[p - 1].s == 'n') {"),
    "pdd_discard_all": ("} else if (p >= 2 && P[p - 1].s == 'n' && P[p - 2].s == 'n') {",
                        "} else if (false) {"),
    "pdd_partner_any_next": ("const bool next = p + 1 < m && uint64_t(P[p + 1].i) == uint64_t(x.i) + h;",
                             "const bool next = p + 1 < m;"),
    "pdd_comparator_div_first": ("      if (a.i % h != b.i % h) return a.i % h < b.i % h;\n      return a.i / h < b.i / h;\n    });\n    if (round",
                                 "      if (a.i / h != b.i / h) return a.i / h < b.i / h;\n      return a.i % h < b.i % h;\n    });\n    if (round"),
    "pdd_rename_no_group": ("N[p] = Item{I[p].second, static_cast<uint32_t>(r0 + run - grp), 'n'};",
                            "N[p] = Item{I[p].second, static_cast<uint32_t>(1 + run), 'n'};"),
    "pdd_unique_one_side": ("N[j].s = (differs_prev && differs_next) ? 'u' : 'n';",
                            "N[j].s = differs_next ? 'u' : 'n';"),
    "opk_order_swapped": ("    if (a % h != b % h) return a % h < b % h;\n    return a / h < b / h;",
                          "    if (a / h != b / h) return a / h < b / h;\n    return a % h < b % h;"),
    "dc3_rank_zero_based": ("    ++rank;\n    if (i % 3 == 1)", "    if (i % 3 == 1)"),
    "dc3_ranks_swapped": ("      r1[i / 3] = rank;\n    else\n      r2[i / 3] = rank;",
                          "      r2[i / 3] = rank;\n    else\n      r1[i / 3] = rank;"),
    "dcx_cover_ignored": ("    if ((dmask >> (i % X)) & 1u) out[i] = ++rank;",
                          "    if ((dmask >> (i % X)) & 1u) out[i] = ++rank; else ++rank;"),
    "brute_signed": ("return std::lexicographical_compare(T + a, T + n, T + b, T + n);",
                     "return std::lexicographical_compare((const signed char*)T + a, "
                     "(const signed char*)T + n, (const signed char*)T + b, "
                     "(const signed char*)T + n);"),
}


def _run_pins(so_path=None, timeout=120):
    """Run the compact pin set in a fresh interpreter (a mutant may not
    terminate; a time-out counts as caught)."""
    cmd = [sys.executable, PINS]
    if so_path:
        cmd.append(str(so_path))
    try:
        r = subprocess.run(cmd, timeout=timeout, capture_output=True, text=True)
    except subprocess.TimeoutExpired:
        return False
    return r.returncode == 0


def test_unmutated_pins_pass():
    assert _run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found"
    mpath = tmp_path / "mutant.cpp"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", str(so), str(mpath)],
                   check=True)
    assert not _run_pins(so, timeout=15), f"mutant {name} survived the pins"


def test_parallel_build_pins_pass():
    """The GNU-parallel build of the oracle (the CPU baseline, and the checker
    of some large GPU tests) passes the same pins as the sequential build."""
    if not os.path.exists(oracle.LIB_PAR):
        oracle.build(parallel=True)
    assert _run_pins(oracle.LIB_PAR)


def test_parallel_build_at_scale():
    """Above the parallel sort's thresholds the parallel build equals the
    pinned sequential build, and the closed forms hold."""
    n = 1 << 22
    t = np.frombuffer(b"ACGT", np.uint8)[np.random.default_rng(21).integers(0, 4, n)]
    assert np.array_equal(oracle.sa(t, parallel=True), oracle.sa(t))
    m = 1 << 20
    assert np.array_equal(oracle.sa(np.full(m, 97, np.uint8), parallel=True),
                          np.arange(m - 1, -1, -1, dtype=np.uint32))
    ab = np.frombuffer(b"ab" * (m // 2), np.uint8)
    want = np.concatenate([np.arange(m - 2, -1, -2), np.arange(m - 1, 0, -2)]).astype(np.uint32)
    assert np.array_equal(oracle.sa(ab, parallel=True), want)


# --------------------------------------------------------------------------
# Index structures from a suffix array: LCP array, BWT of text$, pattern
# intervals. Expected values come from Python brute force (rotation sorting for
# the BWT, direct comparison, occurrence counting) and closed forms.

from oracle_pins import py_bwt, py_interval, py_lcp  # noqa: E402


def test_index_textbook_banana():
    sa = oracle.sa(b"banana")
    assert oracle.lcp(b"banana", sa).tolist() == [0, 1, 3, 0, 0, 2]
    bw, d = oracle.bwt(b"banana", sa)
    assert bw.tobytes() == b"annbaa" and d == 4  # banana$ -> annb$aa
    assert oracle.sa_interval(b"banana", sa, b"ana") == (1, 3)
    assert oracle.sa_interval(b"banana", sa, b"") == (0, 6)
    assert oracle.sa_interval(b"banana", sa, b"nax") == (6, 6)
    assert oracle.sa_interval(b"banana", sa, b"b") == (3, 4)


@pytest.mark.parametrize("sigma", [1, 2, 4, 256])
def test_index_brute_force(sigma):
    rng = np.random.default_rng(300 + sigma)
    for _ in range(40):
        n = int(rng.integers(1, 90))
        t = rng.integers(0, sigma, n).astype(np.uint8)
        tb = t.tobytes()
        sa = oracle.sa(t)
        assert oracle.lcp(t, sa).tolist() == py_lcp(tb)
        bw, d = oracle.bwt(t, sa)
        assert (bw.tobytes(), d) == py_bwt(tb)
        for _ in range(5):
            a = int(rng.integers(0, n))
            pat = tb[a:a + int(rng.integers(0, 5))]
            assert oracle.sa_interval(t, sa, pat) == py_interval(tb, pat)
            pat = rng.integers(0, sigma, int(rng.integers(1, 4))).astype(np.uint8).tobytes()
            assert oracle.sa_interval(t, sa, pat) == py_interval(tb, pat)


def test_index_closed_forms():
    n = 2000
    a = np.full(n, 97, np.uint8)
    sa = oracle.sa(a)
    assert oracle.lcp(a, sa).tolist() == list(range(n))          # a^j vs a^(j+1)
    bw, d = oracle.bwt(a, sa)
    assert bw.tobytes() == b"a" * n and d == n                     # $ ends the column
    assert oracle.sa_interval(a, sa, b"a" * 10) == (9, n)        # suffixes a^10 .. a^n
    m = 500
    ab = np.frombuffer(b"ab" * m, np.uint8)
    sa = oracle.sa(ab)
    # (ab)^m: SA lists the a-suffixes (ab)^k, k = 1..m, then the b-suffixes
    # b(ab)^k, k = 0..m-1; each neighbour shares all of the shorter suffix:
    # (ab)^k with (ab)^(k+1) 2k bytes, b(ab)^(k-1) with b(ab)^k 2k - 1 bytes.
    want = [0] + [2 * k for k in range(1, m)] + [0] + [2 * k - 1 for k in range(1, m)]
    assert oracle.lcp(ab, sa).tolist() == want
    bw, d = oracle.bwt(ab, sa)
    assert bw.tobytes() == b"b" + b"b" * (m - 1) + b"a" * m and d == m
