"""GPU parity of the difference cover algorithm DC7 (Section 2.2): the sample
is positions 0, 1, 3 mod 7; the suffix array must equal the oracle's bit for
bit, and the sample ranks by position the oracle's by-definition ranks. Texts
cover every length mod 7 (a dummy ends the first part when n mod 7 == 0, the
second when n mod 7 == 1), texts whose sample tuples repeat (recursion through
DC3, with two-word levels at the larger sizes) and NUL bytes."""

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


def check(builder, text, ranks=True, parallel=False):
    t = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    sa, rk = builder.build_dc7(dev(t), with_ranks=True)
    torch.cuda.synchronize()
    got = sa.cpu().numpy().view(np.uint32)
    info = builder.last_info()
    want = oracle.sa(t, parallel=parallel)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"n={t.size}: {bad.size} mismatches, first at {bad[:5].tolist()}; "
                             f"levels={info['rounds']}")
    if ranks and t.size:
        assert np.array_equal(rk.cpu().numpy().view(np.uint32),
                              oracle.dcx_sample_ranks(t, 7, (0, 1, 3)))
    return info


def test_empty(builder):
    assert builder.build_dc7(torch.empty(0, dtype=torch.uint8, device="cuda:0")).numel() == 0


@pytest.mark.parametrize("text", [b"x", b"ab", b"ba", b"aa", b"aaa", b"aba", b"a\0\0",
                                  b"\0\0\0\0", b"banana", b"bdacbdacb", b"dbacbacbd",
                                  bytes(range(256)), bytes(range(255, -1, -1)),
                                  bytes(range(256)) * 3])
def test_small_edge_texts(builder, text):
    check(builder, text)


@pytest.mark.parametrize("n", list(range(1, 16)) + [49, 50, 51, 2049, 4097, 100000])
def test_unary(builder, n):
    """a^n for every n mod 7: every tuple repeats, so the name string recurses."""
    check(builder, b"a" * n)


@pytest.mark.parametrize("m", [1, 7, 1000, 5000])
def test_ab_repeats(builder, m):
    check(builder, b"ab" * m)


@pytest.mark.parametrize("sigma", [1, 2, 4, 96, 256])
def test_random_small(builder, sigma):
    rng = np.random.default_rng(9000 + sigma)
    for _ in range(40):
        n = int(rng.integers(1, 700))
        check(builder, rng.integers(0, sigma, n).astype(np.uint8))


@pytest.mark.parametrize("n", [4095, 4096, 4097, 12289, 65537, 200003])
@pytest.mark.parametrize("kind", ["dna", "binary", "markov", "bytes"])
def test_random_tiles(builder, n, kind):
    rng = np.random.default_rng(n + 29)
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
    rng = np.random.default_rng(31)
    for t in (np.tile(rng.integers(0, 4, 17).astype(np.uint8), 3000),
              np.tile(rng.integers(0, 4, 7).astype(np.uint8), 3000),
              W.repetitive(copies=64, base_len=4096), W.repetitive(copies=20, base_len=3001)):
        check(builder, t)


def test_large(builder):
    """2^23 binary bytes (the name string of 3.6e6 symbols recurses through
    DC3 with two-word levels) and 2^24 bytes of Markov text."""
    rng = np.random.default_rng(37)
    t = rng.integers(0, 2, 1 << 23).astype(np.uint8)
    info = check(builder, t, parallel=True)
    assert info["rounds"] >= 2
    check(builder, W.markov3(1 << 24, chain_seed=37), ranks=False, parallel=True)
