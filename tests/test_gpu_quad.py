"""GPU parity of prefix quadrupling (Section 2.1, "Prefix Quadrupling"): later
rounds sort rank quadruples (ISA[i], ISA[i+h], ISA[i+2h], ISA[i+3h]) and resolve
four times the prefix length per round. The suffix array is unique, so it must
equal the oracle's bit for bit; after every round the names must equal the
closed form 1 + #{j : pad_h(j) < pad_h(i)} at the prefix length that round
resolves (c * 4^k after round k, c characters in round 0)."""

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
    b.set_tuning(prefix_mult=4)
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


def assert_same(builder, text, parallel=False):
    t = np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text
    want = oracle.sa(t, parallel=parallel)
    got = gpu_sa(builder, t)
    info = builder.last_info()
    assert builder.tuning()["prefix_mult"] == 4
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"n={t.size}: {bad.size} mismatches, first at {bad[:5].tolist()}; "
                             f"info={info}")
    return info


@pytest.mark.parametrize("text", [b"x", b"ab", b"ba", b"aa", b"a\0\0", b"\0\0\0\0", b"banana",
                                  b"bdacbdacb", b"dbacbacbd", bytes(range(256)),
                                  bytes(range(255, -1, -1)), bytes(range(256)) * 3])
def test_small_edge_texts(builder, text):
    assert_same(builder, text)


@pytest.mark.parametrize("n", [2, 65, 2049, 4097, 70000])
def test_unary(builder, n):
    """a^n: every round keeps all but the shortest suffixes; the most rounds."""
    assert gpu_sa(builder, b"a" * n).tolist() == list(range(n - 1, -1, -1))


@pytest.mark.parametrize("m", [1, 7, 1000, 5000])
def test_ab_repeats(builder, m):
    want = list(range(2 * m - 2, -1, -2)) + list(range(2 * m - 1, 0, -2))
    assert gpu_sa(builder, b"ab" * m).tolist() == want


@pytest.mark.parametrize("sigma", [1, 2, 4, 96, 256])
def test_random_small(builder, sigma):
    rng = np.random.default_rng(3000 + sigma)
    for _ in range(30):
        n = int(rng.integers(1, 600))
        assert_same(builder, rng.integers(0, sigma, n).astype(np.uint8))


@pytest.mark.parametrize("n", [4095, 4097, 12289, 65537, 200003])
@pytest.mark.parametrize("kind", ["dna", "binary", "markov"])
def test_random_tiles(builder, n, kind):
    rng = np.random.default_rng(n + 7)
    if kind == "dna":
        t = W.dna(n, seed=n)
    elif kind == "binary":
        t = rng.integers(0, 2, n).astype(np.uint8)
    else:
        t = W.markov3(n, chain_seed=n)
    assert_same(builder, t)


def test_repetitive_and_periodic(builder):
    """Texts that keep most suffixes active for many rounds (dense rounds, then
    list rounds on the survivors)."""
    rng = np.random.default_rng(9)
    for t in (W.repetitive(copies=64, base_len=4096), W.repetitive(copies=20, base_len=3001),
              np.tile(rng.integers(0, 4, 17).astype(np.uint8), 3000)):
        info = assert_same(builder, t)
        assert info["key_bits"][1] == 4 * int(t.size).bit_length()


@pytest.mark.parametrize("kind", ["dna", "markov", "repetitive", "binary", "unary"])
def test_round_names_closed_form(builder, kind):
    """After round k the names equal the closed form at prefix length c * 4^k,
    discarded suffixes included."""
    n = 20000
    if kind == "dna":
        t = W.dna(n, seed=5)
    elif kind == "markov":
        t = W.markov3(n, chain_seed=5)
    elif kind == "repetitive":
        t = W.repetitive(copies=10, base_len=2000)
    elif kind == "unary":
        t = np.full(5000, 7, np.uint8)
    else:
        t = np.random.default_rng(5).integers(0, 2, n).astype(np.uint8)
    _, _, full = builder.build_rounds(dev(t), 0)
    c = full["chars0"]
    for k in range(1, full["rounds"] + 1):
        _, isa, info = builder.build_rounds(dev(t), k)
        assert info["rounds"] == k
        assert info["prefix_len"] == c * 4 ** (k - 1)
        want = oracle.prefix_ranks(t, info["prefix_len"])
        assert np.array_equal(isa.cpu().numpy().view(np.uint32), want), (kind, k, info)


def test_fewer_rounds_than_doubling(builder):
    """Same suffix array in about half the later rounds of doubling."""
    t = W.repetitive(copies=48, base_len=8192)
    quad = assert_same(builder, t, parallel=True)
    builder.set_tuning(prefix_mult=2)
    try:
        sa2 = gpu_sa(builder, t)
        dbl = builder.last_info()
    finally:
        builder.set_tuning(prefix_mult=4)
    assert np.array_equal(sa2, oracle.sa(t, parallel=True))
    assert quad["rounds"] - 1 <= (dbl["rounds"] - 1 + 1) // 2 + 1, (quad["rounds"], dbl["rounds"])


@pytest.mark.parametrize("ahead,graphs", [(1, 1), (3, 0), (0, 0)])
def test_rounds_ahead_and_graph_replays(builder, ahead, graphs):
    """Quadrupling rounds run ahead of the host and replay from captured graphs
    (two sorts per round, the second reading its count from the first)."""
    t = W.repetitive(copies=30, base_len=5003)
    want = oracle.sa(t)
    builder.set_tuning(prefix_mult=4, rounds_ahead=ahead, round_graphs=graphs)
    try:
        for _ in range(4):
            assert np.array_equal(gpu_sa(builder, t), want)
    finally:
        builder.set_tuning(prefix_mult=4, rounds_ahead=0, round_graphs=0)


def test_sixteen_mib_repetitive(builder):
    """2^24 bytes of 64 KiB copies with rare substitutions: dense quadrupling
    rounds at a size where the sort spans many chunks; element by element
    against the parallel oracle."""
    t = W.repetitive(copies=256, base_len=1 << 16)
    info = assert_same(builder, t, parallel=True)
    print(f"rounds={info['rounds']} active={info['active']}", flush=True)
