"""GPU parity of prefix doubling with discarding by sorting (Section 2.1,
Alg. 5 with the comparator of Eq. 1 and Alg. 6's Unique / NPairs / renaming):
no inverse suffix array; pairs come from neighbours in the comparator's order.

The suffix array is unique, so it must equal the oracle's bit for bit. Which
items a round sorts, pairs, discards and keeps is fixed by the method too, so
the per-round counts (|P|, |I|, discarded, kept) must equal the oracle's own
run of Alg. 5 from the same first prefix length (the GPU's round-0 width)."""

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def builder():
    from paper_1610_03007_amd import SuffixArrayBuilder
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    b = SuffixArrayBuilder(0, tune_cache="")
    yield b
    b.close()


def dev(a) -> torch.Tensor:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check(builder, text, counts_too=True, parallel=False):
    t = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    sa, counts = builder.build_sorted_pairs(dev(t))
    torch.cuda.synchronize()
    got = sa.cpu().numpy().view(np.uint32)
    info = builder.last_info()
    want = oracle.sa(t, parallel=parallel)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"n={t.size}: {bad.size} mismatches, first at {bad[:5].tolist()}; "
                             f"info={info}")
    if counts_too and t.size:
        ref_sa, ref_counts = oracle.pdd_sa(t, info["chars0"])
        assert np.array_equal(ref_sa, want)
        assert counts.astype(np.int64).tolist() == ref_counts.astype(np.int64).tolist(), \
            (counts.tolist(), ref_counts.tolist())
    return info, counts


def test_empty(builder):
    sa, counts = builder.build_sorted_pairs(torch.empty(0, dtype=torch.uint8, device="cuda:0"))
    assert sa.numel() == 0 and counts.shape[0] == 0


@pytest.mark.parametrize("text", [b"x", b"ab", b"ba", b"aa", b"aba", b"a\0\0", b"\0\0\0\0",
                                  b"banana", b"bdacbdacb", b"dbacbacbd", bytes(range(256)),
                                  bytes(range(255, -1, -1)), bytes(range(256)) * 3])
def test_small_edge_texts(builder, text):
    check(builder, text)


@pytest.mark.parametrize("n", [2, 65, 2049, 4097, 30000])
def test_unary(builder, n):
    info, _ = check(builder, b"a" * n)
    assert info["rounds"] >= 2


@pytest.mark.parametrize("m", [1, 7, 1000, 5000])
def test_ab_repeats(builder, m):
    check(builder, b"ab" * m)


@pytest.mark.parametrize("sigma", [1, 2, 4, 96, 256])
def test_random_small(builder, sigma):
    rng = np.random.default_rng(5000 + sigma)
    for _ in range(30):
        n = int(rng.integers(1, 600))
        check(builder, rng.integers(0, sigma, n).astype(np.uint8))


@pytest.mark.parametrize("n", [4095, 4097, 12289, 65537, 200003])
@pytest.mark.parametrize("kind", ["dna", "binary", "markov"])
def test_random_tiles(builder, n, kind):
    rng = np.random.default_rng(n + 11)
    if kind == "dna":
        t = W.dna(n, seed=n)
    elif kind == "binary":
        t = rng.integers(0, 2, n).astype(np.uint8)
    else:
        t = W.markov3(n, chain_seed=n)
    check(builder, t)


def test_repetitive_and_periodic(builder):
    rng = np.random.default_rng(13)
    for t in (W.repetitive(copies=64, base_len=4096), W.repetitive(copies=20, base_len=3001),
              np.tile(rng.integers(0, 4, 17).astype(np.uint8), 3000)):
        info, counts = check(builder, t)
        # Kept items are few next to the items sorted.
        assert counts[:, 3].sum() <= counts[:, 0].sum()


def test_digit_widths(builder):
    """The comparator keys and the name pairs sort at every digit width."""
    t = W.repetitive(copies=16, base_len=5000)
    for rb, items in ((6, 8), (7, 8), (9, 8), (8, 8)):
        builder.set_tuning(radix_bits=rb, sort_items=items, sort_block=512, sort_match=0)
        try:
            check(builder, t)
        finally:
            builder.auto_tuning()


def test_two_mib_markov_and_dna(builder):
    """2^21-byte texts: several sort chunks per round; element by element
    against the parallel oracle, and counts against Alg. 5."""
    for t in (W.markov3(1 << 21, chain_seed=21), W.dna(1 << 21, seed=21)):
        info, counts = check(builder, t, parallel=True)
        print(f"n={t.size} rounds={info['rounds']} counts={counts.tolist()}", flush=True)
