"""GPU parity of the batched build: every text's suffix array from one batched
build equals the oracle's suffix array of that text alone (bit-exact)."""

import concurrent.futures as cf

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
    b = SuffixArrayBuilder(0)
    yield b
    b.close()


def run_batch(builder, texts):
    lengths = [t.size for t in texts]
    off = np.zeros(len(texts) + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    cat = np.concatenate(texts) if texts else np.zeros(0, np.uint8)
    d = torch.from_numpy(cat.copy()).to("cuda:0")
    sa = builder.build_batch(d, off)
    torch.cuda.synchronize()
    return sa.cpu().numpy().view(np.uint32), off


def check_each(texts, sa, off):
    for t, text in enumerate(texts):
        got = sa[int(off[t]):int(off[t + 1])]
        want = oracle.sa(text)
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0]
            raise AssertionError(f"text {t} (n={text.size}): {bad.size} mismatches, first {bad[:5]}")


def mixed_texts(rng, count, max_len):
    texts = []
    for i in range(count):
        n = int(rng.choice([0, 1, 2, 3, int(rng.integers(4, max_len))]))
        kind = i % 4
        if kind == 0:
            t = W.dna(n, seed=int(rng.integers(1 << 30)))
        elif kind == 1:
            t = W.markov3(n, chain_seed=int(rng.integers(1 << 30)))
        elif kind == 2:
            t = rng.integers(0, 2, n).astype(np.uint8)
        else:
            t = rng.integers(0, 256, n).astype(np.uint8)
        texts.append(np.ascontiguousarray(t, dtype=np.uint8))
    return texts


@pytest.mark.parametrize("count,max_len,seed", [(2, 50, 0), (7, 300, 1), (60, 3000, 2),
                                                (300, 2000, 3), (2500, 200, 4)])
def test_batch_matches_oracle(builder, count, max_len, seed):
    rng = np.random.default_rng(seed)
    texts = mixed_texts(rng, count, max_len)
    sa, off = run_batch(builder, texts)
    check_each(texts, sa, off)
    info = builder.last_info()
    assert info["n"] == int(off[-1])


def test_batch_repetitive_and_unary(builder):
    texts = [b"a" * 5000, b"ab" * 3000, W.repetitive(copies=20, base_len=1500),
             bytes(range(256)) * 4, b"", b"z"]
    texts = [np.frombuffer(bytes(t), np.uint8) if isinstance(t, bytes) else t for t in texts]
    sa, off = run_batch(builder, texts)
    check_each(texts, sa, off)


@pytest.mark.parametrize("mode", ["eager", "lazy", "auto"])
def test_batch_isa_modes(builder, mode):
    """The ISA after round 0 formed eagerly (every name scattered) or lazily
    (survivors only; other names recomputed by a search in the text's own
    range of round-0 sorted keys) gives the same arrays. Repetitive texts keep
    suffixes alive for many rounds, so lazy gathers reach both forms of name;
    the empty and one-symbol texts check the text ranges at the edges."""
    rng = np.random.default_rng(21)
    # About 20k suffixes, of which about 4.5k survive round 0 (the forced lazy
    # form needs at most a third).
    texts = [W.repetitive(copies=6, base_len=300), b"", b"q", b"ab" * 400,
             W.dna(5000, seed=3), b"a" * 600, rng.integers(0, 3, 4000).astype(np.uint8),
             W.markov3(7000, chain_seed=5), b"", W.repetitive(copies=20, base_len=60)]
    texts = [np.frombuffer(bytes(t), np.uint8) if isinstance(t, bytes) else
             np.ascontiguousarray(t, np.uint8) for t in texts]
    builder.set_isa_mode(mode)
    try:
        sa, off = run_batch(builder, texts)
        info = builder.last_info()
    finally:
        builder.set_isa_mode("auto")
    check_each(texts, sa, off)
    assert info["rounds"] >= 3
    if mode == "eager":
        assert info["lazy_isa"] == 0
    elif mode == "lazy":
        assert info["lazy_isa"] == 1


@pytest.mark.parametrize("match", [0, 1])
def test_batch_digit_match(builder, match):
    """Both sweep digit matches on multi-text keys (slot bits on top)."""
    rng = np.random.default_rng(40 + match)
    texts = mixed_texts(rng, 200, 5000)
    builder.set_tuning(sort_match=match, radix_bits=8, sort_items=8, sort_block=512)
    try:
        sa, off = run_batch(builder, texts)
        assert builder.tuning()["sort_match"] == match
    finally:
        builder.auto_tuning()
    check_each(texts, sa, off)


def test_batch_lazy_at_scale(builder):
    """Many Markov and DNA texts (2^24 suffixes in all): few suffixes survive
    round 0, so the automatic choice is the lazy ISA."""
    rng = np.random.default_rng(33)
    texts, total = [], 0
    i = 0
    while total < (1 << 24):
        n = int(rng.integers(1 << 12, 1 << 18))
        t = W.markov3(n, chain_seed=100 + i) if i % 2 == 0 else W.dna(n, seed=100 + i)
        texts.append(np.ascontiguousarray(t, np.uint8))
        total += n
        i += 1
    sa, off = run_batch(builder, texts)
    info = builder.last_info()
    assert info["lazy_isa"] == 1
    for t in range(0, len(texts), 7):
        got = sa[int(off[t]):int(off[t + 1])]
        assert np.array_equal(got, oracle.sa(texts[t])), f"text {t}"


def test_batch_equals_single_builds(builder):
    """The batched path and one build per text give identical arrays."""
    rng = np.random.default_rng(9)
    texts = mixed_texts(rng, 40, 20000)
    sa, off = run_batch(builder, texts)
    for t, text in enumerate(texts):
        if text.size == 0:
            continue
        single = builder.build(torch.from_numpy(text.copy()).to("cuda:0"))
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy().view(np.uint32), sa[int(off[t]):int(off[t + 1])])


@pytest.mark.parametrize("round0_full", [0, 1])
def test_batch_round0_layout(builder, round0_full):
    """100 DNA and Markov texts (7 slot bits) with 8-bit digits: with round-0
    trimming the slot sits right above the characters, which take at most
    56 - 7 = 49 bits, so round 0 runs at most 7 sweeps; without it the slot
    takes the top bits of 64-bit keys (8 sweeps). Both layouts give the same
    arrays."""
    rng = np.random.default_rng(77)
    texts = []
    for i in range(100):
        n = int(rng.integers(1, 40000))
        t = W.dna(n, seed=300 + i) if i % 2 else W.markov3(n, chain_seed=300 + i)
        texts.append(np.ascontiguousarray(t, np.uint8))
    builder.set_tuning(round0_full=round0_full, radix_bits=8, sort_items=8, sort_block=512)
    try:
        sa, off = run_batch(builder, texts)
        info = builder.last_info()
    finally:
        builder.auto_tuning()
    check_each(texts, sa, off)
    if round0_full:
        assert info["passes_run"][0] == 8, info["passes_run"][:2]
    else:
        assert info["passes_run"][0] <= 7, info["passes_run"][:2]


def test_batch_errors(builder):
    from paper_1610_03007_amd import SAError
    d = torch.zeros(10, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(SAError):
        builder.build_batch(d, [1, 5, 10])        # offsets[0] != 0
    with pytest.raises(SAError):
        builder.build_batch(d, [0, 6, 5, 10])     # decreasing
    with pytest.raises(ValueError):
        builder.build_batch(d, [0, 5])            # does not cover the text


def test_batch_full_size(builder):
    """4096 texts, lengths log-uniform in [4 KiB, 8 MiB], alternating DNA and
    Markov (the batched workload at full size, total about 4.5e9 bytes): one
    batched build; every text's array passes the oracle's linear-time check
    and a sample of texts is compared with the oracle element by element."""
    texts, off = W.batch()
    n_total = int(off[-1])
    assert n_total > (1 << 32)
    d = torch.from_numpy(texts).to("cuda:0")
    sa_d = builder.build_batch(d, off)
    torch.cuda.synchronize()
    info = builder.last_info()
    assert info["n"] == n_total
    del d
    sa = sa_d.cpu().numpy().view(np.uint32)
    del sa_d
    torch.cuda.empty_cache()

    def check(t):
        a, b = int(off[t]), int(off[t + 1])
        return t, oracle.check_sa(texts[a:b], sa[a:b])

    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        for t, (status, where) in ex.map(check, range(off.size - 1)):
            assert status == 0, (t, status, where)
    rng = np.random.default_rng(0)
    lengths = np.diff(off.astype(np.int64))
    small = np.nonzero(lengths < 200000)[0]
    for t in rng.choice(small, 16, replace=False):
        a, b = int(off[t]), int(off[t + 1])
        assert np.array_equal(sa[a:b], oracle.sa(texts[a:b])), t


@pytest.mark.parametrize("mode", ["auto", "eager"])
def test_batch_full_64bit_keys(builder, mode):
    """4096 texts whose longest has 2^25..2^26 bytes: 12 slot bits plus two
    26-bit ranks fill all 64 key bits, and the long text takes the last slot
    (every slot bit set)."""
    rng = np.random.default_rng(64)
    texts = []
    for i in range(4095):
        n = int(rng.integers(0, 300))
        texts.append(W.dna(n, seed=i) if i % 2 else
                     rng.integers(0, 256, n).astype(np.uint8))
    big = W.markov3((1 << 25) + 12345, chain_seed=64)
    big[-4096:] = big[:4096]  # a repeat: the long text needs more rounds
    texts.append(big)
    builder.set_isa_mode(mode)
    try:
        sa, off = run_batch(builder, texts)
    finally:
        builder.set_isa_mode("auto")
    assert len(texts) == 4096 and 12 + 2 * 26 == 64
    assert np.array_equal(sa[int(off[-2]):int(off[-1])], oracle.sa(big, parallel=True))
    check_each(texts[:-1], sa, off)
