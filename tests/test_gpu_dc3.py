"""GPU parity of the difference cover algorithm DC3 (Section 2.2, Alg. 7).

The suffix array is unique, so it must equal the oracle's bit for bit; the
top level's sample ranks (the suffixes at positions i mod 3 != 0 ranked among
themselves) must equal the oracle's by-definition ranks, and Example 3's
printed R1/R2. Texts cover every length mod 3 (the dummy sample position when
n mod 3 == 1), unary and periodic texts (deep recursion), NUL bytes, and sizes
whose reduced strings need two-word triple sorts (names of more than 21 bits)."""

import json
import math
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
    b = SuffixArrayBuilder(0, tune_cache="")
    yield b
    b.close()


def dev(a) -> torch.Tensor:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def check(builder, text, ranks=True, parallel=False):
    t = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    sa, r12 = builder.build_dc3(dev(t), with_ranks=True)
    torch.cuda.synchronize()
    got = sa.cpu().numpy().view(np.uint32)
    info = builder.last_info()
    want = oracle.sa(t, parallel=parallel)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"n={t.size}: {bad.size} mismatches, first at {bad[:5].tolist()}; "
                             f"levels={info['rounds']}")
    if ranks and t.size:
        r = r12.cpu().numpy().view(np.uint32)
        r1, r2 = oracle.dc3_sample_ranks(t)
        assert np.array_equal(r[1::3], r1) and np.array_equal(r[2::3], r2)
        assert not r[0::3].any()
    return info


def test_example3(builder):
    g = json.load(open(os.path.join(GOLDEN, "paper_example3_dbacbacbd.json")))
    sa, r12 = builder.build_dc3(dev(g["text"].encode()), with_ranks=True)
    torch.cuda.synchronize()
    assert sa.cpu().numpy().tolist() == g["sa"]
    r = r12.cpu().numpy().tolist()
    assert r[1::3] == g["dc3_r1"] and r[2::3] == g["dc3_r2"]


def test_empty(builder):
    sa = builder.build_dc3(torch.empty(0, dtype=torch.uint8, device="cuda:0"))
    assert sa.numel() == 0


@pytest.mark.parametrize("text", [b"x", b"ab", b"ba", b"aa", b"aaa", b"aba", b"a\0\0",
                                  b"\0\0\0\0", b"banana", b"bdacbdacb", bytes(range(256)),
                                  bytes(range(255, -1, -1)), bytes(range(256)) * 3])
def test_small_edge_texts(builder, text):
    check(builder, text)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 64, 65, 66, 2049, 4097, 100000])
def test_unary(builder, n):
    """a^n: every level's triples repeat, so the recursion goes on until the
    runs of equal names (a third as long at each level) are short."""
    info = check(builder, b"a" * n)
    if n > 1000:
        assert info["rounds"] >= int(math.log(n, 3)) - 1, info["rounds"]


@pytest.mark.parametrize("m", [1, 7, 1000, 5000])
def test_ab_repeats(builder, m):
    check(builder, b"ab" * m)


@pytest.mark.parametrize("sigma", [1, 2, 4, 96, 256])
def test_random_small(builder, sigma):
    rng = np.random.default_rng(7000 + sigma)
    for _ in range(40):
        n = int(rng.integers(1, 700))
        check(builder, rng.integers(0, sigma, n).astype(np.uint8))


@pytest.mark.parametrize("n", [4095, 4096, 4097, 12289, 65537, 200003])
@pytest.mark.parametrize("kind", ["dna", "binary", "markov", "bytes"])
def test_random_tiles(builder, n, kind):
    rng = np.random.default_rng(n + 17)
    if kind == "dna":
        t = W.dna(n, seed=n)
    elif kind == "binary":
        t = rng.integers(0, 2, n).astype(np.uint8)
    elif kind == "bytes":
        t = rng.integers(0, 256, n).astype(np.uint8)
    else:
        t = W.markov3(n, chain_seed=n)
    check(builder, t)


def test_periodic_and_repetitive(builder):
    rng = np.random.default_rng(19)
    for t in (np.tile(rng.integers(0, 4, 17).astype(np.uint8), 3000),
              W.repetitive(copies=64, base_len=4096), W.repetitive(copies=20, base_len=3001)):
        check(builder, t)


def test_two_word_triples(builder):
    """Reduced strings longer than 2^21 name their triples with more than 21
    bits, so those levels sort triples as two words: a 2^23-byte binary text
    (its first reduced string has about 5.6e6 symbols) and 2^22 periodic
    bytes (deep recursion on long reduced strings)."""
    rng = np.random.default_rng(23)
    t = rng.integers(0, 2, 1 << 23).astype(np.uint8)
    info = check(builder, t, parallel=True)
    assert info["active"][1] > (1 << 21)
    u = np.tile(rng.integers(0, 4, 5).astype(np.uint8), (1 << 22) // 5)
    check(builder, u, ranks=False, parallel=True)


def test_markov_16mib(builder):
    t = W.markov3(1 << 24, chain_seed=24)
    info = check(builder, t, ranks=False, parallel=True)
    print(f"levels={info['rounds']} sizes={info['active'][:info['rounds']]}", flush=True)
