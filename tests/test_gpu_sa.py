"""GPU parity: the HIP suffix-array path against the CPU oracle.

Bit-exact comparison (the suffix array is unique and all arithmetic is
integer). Small and medium texts are compared element by element with
``oracle.sa``; per-round names with the oracle's closed form; the full-size
256 MiB and 1 GiB texts with the oracle's linear-time suffix-array check plus
sampled direct suffix comparisons.
"""

import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def builder():
    from paper_1610_03007_amd import SuffixArrayBuilder
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    b = SuffixArrayBuilder(0)
    yield b
    b.close()


def dev(a) -> torch.Tensor:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_sa(builder, text) -> np.ndarray:
    sa = builder.build(dev(text))
    torch.cuda.synchronize()
    return sa.cpu().numpy().view(np.uint32)


def assert_same(builder, text):
    t = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    want = oracle.sa(t)
    got = gpu_sa(builder, t)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"n={t.size}: {bad.size} mismatches, first at {bad[:5].tolist()}; "
                             f"info={builder.last_info()}")


@pytest.mark.parametrize("fixture", ["paper_example1_bdacbdacb.json",
                                     "paper_example3_dbacbacbd.json", "banana.json"])
def test_golden(builder, fixture):
    g = json.load(open(os.path.join(GOLDEN, fixture)))
    assert gpu_sa(builder, g["text"].encode()).tolist() == g["sa"]


def test_empty(builder):
    sa = builder.build(torch.empty(0, dtype=torch.uint8, device="cuda:0"))
    assert sa.numel() == 0


@pytest.mark.parametrize("text", [b"x", b"ab", b"ba", b"aa", b"a\0\0", b"\0\0\0\0",
                                  b"\0a\0a\0", bytes(range(256)), bytes(range(255, -1, -1)),
                                  bytes(range(256)) * 3])
def test_small_edge_texts(builder, text):
    assert_same(builder, text)


@pytest.mark.parametrize("n", [2, 63, 64, 65, 2047, 2048, 2049, 4095, 4096, 4097, 70000])
def test_unary(builder, n):
    assert gpu_sa(builder, b"a" * n).tolist() == list(range(n - 1, -1, -1))


@pytest.mark.parametrize("m", [1, 7, 1000, 5000])
def test_ab_repeats(builder, m):
    want = list(range(2 * m - 2, -1, -2)) + list(range(2 * m - 1, 0, -2))
    assert gpu_sa(builder, b"ab" * m).tolist() == want


@pytest.mark.parametrize("sigma", [1, 2, 3, 4, 96, 255, 256])
def test_random_small(builder, sigma):
    rng = np.random.default_rng(1000 + sigma)
    for _ in range(40):
        n = int(rng.integers(1, 600))
        t = rng.integers(0, sigma, n).astype(np.uint8)
        assert_same(builder, t)


@pytest.mark.parametrize("n", [4095, 4096, 4097, 8191, 12289, 65537, 200003])
@pytest.mark.parametrize("kind", ["dna", "binary", "bytes", "markov"])
def test_random_tiles(builder, n, kind):
    rng = np.random.default_rng(n)
    if kind == "dna":
        t = W.dna(n, seed=n)
    elif kind == "binary":
        t = rng.integers(0, 2, n).astype(np.uint8)
    elif kind == "bytes":
        t = rng.integers(0, 256, n).astype(np.uint8)
    else:
        t = W.markov3(n, chain_seed=n)
    assert_same(builder, t)


def test_periodic_texts(builder):
    rng = np.random.default_rng(5)
    for period in (3, 17, 1000):
        unit = rng.integers(0, 4, period).astype(np.uint8)
        t = np.tile(unit, 50000 // period + 1)[:50000]
        assert_same(builder, t)


def test_repetitive_small(builder):
    assert_same(builder, W.repetitive(copies=64, base_len=4096))


@pytest.mark.parametrize("kind", ["dna", "markov", "repetitive", "binary"])
def test_round_names_closed_form(builder, kind):
    """After every round k, ISA equals 1 + #{j : pad_h(j) < pad_h(i)} for the
    prefix length h that round resolves (discarded suffixes included)."""
    n = 20000
    if kind == "dna":
        t = W.dna(n, seed=3)
    elif kind == "markov":
        t = W.markov3(n, chain_seed=3)
    elif kind == "repetitive":
        t = W.repetitive(copies=10, base_len=2000)
    else:
        t = np.random.default_rng(3).integers(0, 2, n).astype(np.uint8)
    _, _, full = builder.build_rounds(dev(t), 0)
    for k in range(1, full["rounds"] + 1):
        _, isa, info = builder.build_rounds(dev(t), k)
        assert info["rounds"] == k
        want = oracle.prefix_ranks(t, info["prefix_len"])
        got = isa.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (kind, k, info)


def two_copy_text(n_rand: int, block: int, seed: int) -> np.ndarray:
    """Random Markov text followed by two copies of one block: about 2*block of
    the suffixes survive round 0."""
    rng = np.random.default_rng(seed)
    base = W.markov3(n_rand, chain_seed=seed)
    blk = W.SYMBOLS96[rng.integers(0, 96, block)]
    return np.concatenate([base, blk, blk])


@pytest.mark.parametrize("mode", ["eager", "lazy", "auto"])
def test_isa_modes(builder, mode):
    """Eager and lazy inverse-suffix-array formation after round 0 give the same
    bit-exact SA, and lazily resolved names match the closed form."""
    builder.set_isa_mode(mode)
    try:
        for text in (two_copy_text(30000, 2500, 1), two_copy_text(9000, 5000, 2),
                     W.markov3(70001, chain_seed=4), W.dna(50000, seed=4),
                     np.random.default_rng(0).integers(0, 2, 40000).astype(np.uint8)):
            assert_same(builder, text)
            info = builder.last_info()
            survivors = info["active"][1] if info["rounds"] > 1 else 0
            if mode == "eager":
                assert not info["lazy_isa"]
            elif mode == "lazy":
                carved = (max(survivors, 1) + 63) // 64 * 64
                assert info["lazy_isa"] == (carved * 3 <= text.size)
        t = two_copy_text(30000, 2500, 3)
        _, _, full = builder.build_rounds(dev(t), 0)
        for k in range(1, full["rounds"] + 1):
            _, isa, info = builder.build_rounds(dev(t), k)
            want = oracle.prefix_ranks(t, info["prefix_len"])
            assert np.array_equal(isa.cpu().numpy().view(np.uint32), want), (mode, k, info)
    finally:
        builder.set_isa_mode("auto")


def test_dna1m(builder):
    """n = 2^20 ACGT text (seed 0): bit-exact against the oracle."""
    t = W.dna(1 << 20, seed=0)
    assert_same(builder, t)  # whatever tuning the cache picks
    builder.set_tuning(round0_full=0, radix_bits=8, sort_items=8, sort_block=512)
    try:
        assert_same(builder, t)
        info = builder.last_info()
        assert info["sigma"] == 4 and info["chars0"] == 18  # 3-bit codes, 54 of 56 key bits
        builder.set_tuning(round0_full=1)
        assert_same(builder, t)
        assert builder.last_info()["chars0"] == 21  # 63 key bits
        builder.set_tuning(round0_full=0, radix_bits=7)
        assert_same(builder, t)
        assert builder.last_info()["chars0"] == 21  # 63 bits are nine whole 7-bit digits
    finally:
        builder.auto_tuning()


@pytest.mark.parametrize("bits", [1, 7, 8, 9, 20, 33, 42, 58, 64])
@pytest.mark.parametrize("count", [1, 100, 4095, 4096, 4097, 100000])
def test_radix_sort_pairs(builder, bits, count):
    rng = np.random.default_rng(bits * 1000 + count)
    hi = np.uint64(1) << np.uint64(bits) if bits < 64 else None
    keys = rng.integers(0, 2**63, count, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, count, dtype=np.uint64)
    if hi is not None:
        keys = keys % hi
    if count > 10:
        keys[: count // 10] = keys[0]  # many equal keys: stability matters
    vals = np.arange(count, dtype=np.uint32)[::-1].copy()
    order = np.argsort(keys, kind="stable")
    k_t = dev(keys.view(np.int64))
    v_t = dev(vals.view(np.int32))
    builder.radix_sort_pairs(k_t, v_t, bits)
    torch.cuda.synchronize()
    assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("low_const_bits", [8, 16, 24, 40])
@pytest.mark.parametrize("count", [5000, 300001])
def test_radix_sort_constant_low_digits(builder, low_const_bits, count):
    """Keys whose lowest digits never vary: the first sweep that runs is above
    digit 1, so its chunk counts come from the fallback histogram."""
    rng = np.random.default_rng(low_const_bits + count)
    tail = np.uint64(0xA5A5A5A5A5A5A5A5) & ((np.uint64(1) << np.uint64(low_const_bits)) -
                                             np.uint64(1))
    keys = (rng.integers(0, 2**(64 - low_const_bits), count, dtype=np.uint64)
            << np.uint64(low_const_bits)) | tail
    keys[::5] = keys[1]  # ties
    vals = rng.integers(0, 2**32, count, dtype=np.uint64).astype(np.uint32)
    order = np.argsort(keys, kind="stable")
    k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
    builder.radix_sort_pairs(k_t, v_t, 64)
    torch.cuda.synchronize()
    assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("bits", [8, 16, 64])
def test_radix_sort_all_equal(builder, bits):
    keys = np.full(50000, 0xC5 if bits == 8 else 12345, dtype=np.uint64)
    vals = np.arange(50000, dtype=np.uint32)
    k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
    builder.radix_sort_pairs(k_t, v_t, bits)
    torch.cuda.synchronize()
    assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals)


def test_errors(builder):
    from paper_1610_03007_amd import SAError
    with pytest.raises(SAError):
        builder.build(dev(b"abc"), sigma=0)
    with pytest.raises(TypeError):
        builder.build(torch.zeros(3, dtype=torch.int32, device="cuda:0"))


def sampled_direct_check(t: np.ndarray, sa: np.ndarray, samples: int = 2000, seed: int = 0):
    """Compare SA[j] and SA[j+1] suffixes byte by byte at random j."""
    rng = np.random.default_rng(seed)
    n = t.size
    tb = t.tobytes()
    for j in rng.integers(0, n - 1, samples):
        a, b = int(sa[j]), int(sa[j + 1])
        L = 64
        while True:
            sa_, sb_ = tb[a:a + L], tb[b:b + L]
            if sa_ != sb_ or a + L >= n or b + L >= n:
                break
            L *= 4
        assert tb[a:a + L] < tb[b:b + L] or (tb[a:a + L] == tb[b:b + L] and n - a < n - b), j


def alphabet_text(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "all_bytes":      # 256 symbols: 9-bit codes, 6 characters per key
        return rng.integers(0, 256, n, dtype=np.uint8)
    if kind == "binary":         # 2 symbols: 2-bit codes, 28 characters per key
        return rng.integers(0, 2, n, dtype=np.uint8) * np.uint8(0xFF)
    if kind == "skewed":         # 0x00 most of the time, some rare bytes
        t = np.zeros(n, np.uint8)
        hits = rng.random(n) < 0.01
        t[hits] = rng.integers(1, 256, int(hits.sum()), dtype=np.uint8)
        return t
    if kind == "unary":          # every round keeps every suffix active
        return np.full(n, 0x41, np.uint8)
    if kind == "dna_repeats":    # 1/8 of the text copied 8 times with rare changes
        base = W.dna(n // 8, seed=seed)
        t = np.tile(base, 8)[:n].copy()
        flips = rng.random(n) < 1e-5
        t[flips] = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, int(flips.sum()))]
        return t
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["all_bytes", "binary", "skewed", "unary", "dna_repeats"])
def test_alphabets_at_scale(builder, kind):
    """2^22-byte texts over unusual alphabets and structures, element by element
    against the oracle (unary: against its closed form)."""
    n = 1 << 22
    t = alphabet_text(kind, n, seed=11)
    sa = gpu_sa(builder, t)
    if kind == "unary":
        assert np.array_equal(sa, np.arange(n - 1, -1, -1, dtype=np.uint32))
    else:
        assert np.array_equal(sa, oracle.sa(t, parallel=True))
    info = builder.last_info()
    assert info["n"] == n


@pytest.mark.parametrize("kind", ["markov_256m", "repetitive_1g"])
def test_full_size(builder, kind):
    """Full-size texts in the benchmark's configuration: linear-time check of
    the whole SA plus sampled direct suffix comparisons."""
    if kind == "markov_256m":
        t = W.markov3(1 << 28, chain_seed=2)
    else:
        t = W.repetitive()
    sa = gpu_sa(builder, t)
    info = builder.last_info()
    status, where = oracle.check_sa(t, sa)
    assert status == 0, (kind, status, where, info)
    sampled_direct_check(t, sa)


@pytest.mark.parametrize("match", [0, 1])
@pytest.mark.parametrize("items,block", [(8, 256), (12, 256), (16, 256), (20, 256), (24, 256),
                                         (4, 512), (8, 512), (12, 512)])
def test_sort_tile_variants(builder, items, block, match):
    """Every radix-sort tile shape, with either digit match, sorts stably and
    builds the same SA."""
    builder.set_tuning(sort_items=items, sort_block=block, sort_match=match, radix_bits=8)
    try:
        rng = np.random.default_rng(items)
        count = 100003
        keys = rng.integers(0, 2**62, count, dtype=np.uint64)
        keys[::7] = keys[3]
        vals = rng.integers(0, 2**31, count, dtype=np.uint32)
        order = np.argsort(keys, kind="stable")
        k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
        builder.radix_sort_pairs(k_t, v_t, 62)
        torch.cuda.synchronize()
        assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys[order])
        assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order])
        assert_same(builder, W.dna(200003, seed=items))
        assert_same(builder, W.repetitive(copies=20, base_len=3001))
    finally:
        builder.auto_tuning()


@pytest.mark.parametrize("items,block,match", [(8, 512, 0), (8, 512, 1), (8, 256, 0)])
def test_radix_sort_skewed_next_digit(builder, items, block, match):
    """2^26 keys whose low digit is 0 or 1 and whose next digit is almost
    always 0: each sweep workgroup counts far more than 65535 elements into
    one (output chunk, next digit) bin, so its 16-bit LDS counts must move to
    the global histogram before they overflow."""
    builder.set_tuning(sort_items=items, sort_block=block, sort_match=match, radix_bits=8)
    try:
        rng = np.random.default_rng(items * block)
        count = 1 << 26
        keys = rng.integers(0, 2, count, dtype=np.uint64)
        rare = rng.random(count) < 1e-3
        keys[rare] |= rng.integers(1, 256, int(rare.sum()), dtype=np.uint64) << np.uint64(8)
        vals = np.arange(count, dtype=np.uint32)
        order = np.argsort(keys, kind="stable")
        k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
        builder.radix_sort_pairs(k_t, v_t, 16)
        torch.cuda.synchronize()
        assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order])
        assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys[order])
    finally:
        builder.auto_tuning()


def test_tuning_rejects_bad_values(builder):
    from paper_1610_03007_amd import SAError
    with pytest.raises(SAError):
        builder.set_tuning(sort_items=10)
    with pytest.raises(SAError):
        builder.set_tuning(sort_items=16, sort_block=512)
    with pytest.raises(SAError):
        builder.set_tuning(lazy_ratio=1)
    assert builder.tuning()["sort_items"] in (8, 12, 16, 20, 24)


def test_above_2_31(builder):
    """A text of 2^31 + 4097 bytes: 32-bit ranks, so round keys use all 64
    bits and SA values pass 2^31. The last MiB repeats the first, which keeps
    about 2^21 suffixes active for about 17 rounds. Checked by the oracle's
    linear-time check and sampled direct suffix comparisons."""
    n = (1 << 31) + 4097
    t = W.dna_long(n, seed=31)
    t[-(1 << 20):] = t[:1 << 20]
    sa = gpu_sa(builder, t)
    info = builder.last_info()
    print(f"n={n} rounds={info['rounds']} active={info['active'][:4]}...", flush=True)
    assert info["n"] == n and info["rounds"] >= 17
    assert int(sa.max()) == n - 1
    status, where = oracle.check_sa(t, sa)
    assert status == 0, (status, where, info)
    sampled_direct_check(t, sa, samples=500)


@pytest.mark.parametrize("rb,items", [(6, 4), (6, 8), (6, 12), (7, 4), (7, 8), (7, 12),
                                      (9, 8)])
def test_digit_widths(builder, rb, items):
    """Every radix digit width sorts stably (pairs against numpy's stable sort,
    keys of 1..64 bits) and builds the same SA as the oracle, single and batched."""
    builder.set_tuning(radix_bits=rb, sort_items=items, sort_block=512, sort_match=0)
    try:
        rng = np.random.default_rng(rb * 100 + items)
        for bits, count in ((64, 100003), (13, 70001), (62, 4096 * 9 + 5), (1, 777)):
            keys = rng.integers(0, 2**63, count, dtype=np.uint64) * np.uint64(2) + \
                rng.integers(0, 2, count, dtype=np.uint64)
            if bits < 64:
                keys %= np.uint64(1) << np.uint64(bits)
            keys[::7] = keys[3]
            vals = rng.integers(0, 2**31, count, dtype=np.uint32)
            order = np.argsort(keys, kind="stable")
            k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
            builder.radix_sort_pairs(k_t, v_t, bits)
            torch.cuda.synchronize()
            assert np.array_equal(k_t.cpu().numpy().view(np.uint64), keys[order]), bits
            assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order]), bits
        for t in (W.dna(200003, seed=rb), W.markov3(150001, chain_seed=rb),
                  W.repetitive(copies=20, base_len=3001), np.full(9000, 65, np.uint8)):
            assert_same(builder, t)
            assert builder.last_info()["passes_run"][0] <= -(-64 // rb)
        info = builder.last_info()
        assert builder.tuning()["radix_bits"] == rb
        texts = [W.dna(int(n), seed=int(n)) for n in rng.integers(1, 30000, 40)]
        off = np.zeros(len(texts) + 1, dtype=np.uint64)
        np.cumsum([t.size for t in texts], out=off[1:])
        sa = builder.build_batch(dev(np.concatenate(texts)), off)
        torch.cuda.synchronize()
        sa = sa.cpu().numpy().view(np.uint32)
        for k, t in enumerate(texts):
            assert np.array_equal(sa[int(off[k]):int(off[k + 1])], oracle.sa(t)), k
        del info
    finally:
        builder.auto_tuning()


@pytest.mark.parametrize("rb,items", [(6, 8), (7, 12), (9, 8)])
def test_digit_width_skewed_next_digit(builder, rb, items):
    """2^25 keys whose next digit is almost always 0 at every width: the 16-bit
    next-pass counts must move to the global histogram before they overflow."""
    builder.set_tuning(radix_bits=rb, sort_items=items, sort_block=512, sort_match=0)
    try:
        rng = np.random.default_rng(rb)
        count = 1 << 25
        keys = rng.integers(0, 2, count, dtype=np.uint64)
        rare = rng.random(count) < 1e-3
        keys[rare] |= rng.integers(1, 1 << rb, int(rare.sum()), dtype=np.uint64) << np.uint64(rb)
        vals = np.arange(count, dtype=np.uint32)
        order = np.argsort(keys, kind="stable")
        k_t, v_t = dev(keys.view(np.int64)), dev(vals.view(np.int32))
        builder.radix_sort_pairs(k_t, v_t, 2 * rb)
        torch.cuda.synchronize()
        assert np.array_equal(v_t.cpu().numpy().view(np.uint32), vals[order])
    finally:
        builder.auto_tuning()
