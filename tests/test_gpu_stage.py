"""GPU parity of the staged ISA writes: in a 2^26-byte repetitive text most
suffixes stay active for many rounds, so the re-rank's names go through the
position buckets (at least 2^22 active suffixes, a text of at least 2^26
bytes). The names after each tested round and the suffix array must equal
those of the direct writes, bit for bit, in doubling and quadrupling rounds;
the finished arrays must pass the oracle's linear check and invert each
other."""

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


@pytest.fixture(scope="module")
def text():
    t = W.repetitive(copies=256, base_len=1 << 18)
    assert t.size == 1 << 26
    return t


@pytest.mark.parametrize("prefix_mult", [2, 4])
def test_staged_names_equal_direct(builder, text, prefix_mult):
    d = torch.from_numpy(text).to("cuda:0")
    try:
        for rounds in (2, 5, 64):
            res = {}
            for direct in (1, 0):
                builder.set_tuning(isa_direct=direct, prefix_mult=prefix_mult)
                sa, isa, info = builder.build_rounds(d, rounds)
                torch.cuda.synchronize()
                res[direct] = (sa, isa, info)
            assert max(res[0][2]["active"][1:]) >= (1 << 22), res[0][2]["active"]
            assert torch.equal(res[0][1], res[1][1]), rounds
            assert torch.equal(res[0][0], res[1][0]), rounds
    finally:
        builder.auto_tuning()
    sa, isa, _ = res[0]
    j = torch.arange(text.size, device="cuda:0", dtype=torch.int64)
    assert torch.equal(isa.long()[sa.long()], j + 1)
    assert oracle.check_sa(text, sa.cpu().numpy().view(np.uint32))[0] == 0


def test_staged_full_build(builder, text):
    """sa_build on the same text with the default (staged) writes equals the
    direct build."""
    d = torch.from_numpy(text).to("cuda:0")
    try:
        builder.set_tuning(isa_direct=1)
        want = builder.build(d)
        builder.set_tuning(isa_direct=0)
        got = builder.build(d)
        torch.cuda.synchronize()
    finally:
        builder.auto_tuning()
    assert torch.equal(got, want)


@pytest.mark.parametrize("mode", ["lazy", "eager"])
def test_staged_with_isa_modes(builder, mode):
    """A 2^26-byte DNA text with planted repeats: about 6e6 suffixes survive
    round 0 (at least 2^22, so the later rounds stage their names), in both
    ISA forms; the lazy one carves the later rounds' buffers out of the spare
    keys. Staged and direct writes give the same arrays, which pass the
    oracle's check."""
    n = 1 << 26
    t = W.dna(n, seed=2626).copy()
    rng = np.random.default_rng(2626)
    for _ in range(3000):
        a, b = (int(x) for x in rng.integers(0, n - 1000, 2))
        t[b:b + 1000] = t[a:a + 1000]
    d = torch.from_numpy(t).to("cuda:0")
    builder.set_isa_mode(mode)
    try:
        out = {}
        for direct in (1, 0):
            builder.set_tuning(isa_direct=direct)
            out[direct] = builder.build(d)
            torch.cuda.synchronize()
            info = builder.last_info()
            assert info["lazy_isa"] == (1 if mode == "lazy" else 0)
            assert info["active"][1] >= (1 << 22), info["active"]
    finally:
        builder.set_isa_mode("auto")
        builder.auto_tuning()
    assert torch.equal(out[0], out[1])
    assert oracle.check_sa(t, out[0].cpu().numpy().view(np.uint32))[0] == 0
