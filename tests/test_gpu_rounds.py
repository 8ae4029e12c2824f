"""GPU tests of the round loop run ahead of the host (Section 2.1, Alg. 5 loop
and its stop when no suffix is left): later rounds are enqueued several at a
time, read their count from the device, and replay from a captured HIP graph
once a build's launch arguments repeat. Every replay must give the same
bit-exact result as direct launches and the oracle, with other work and host
synchronisations between the replays."""

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def builder():
    from paper_1610_03007_amd import SuffixArrayBuilder
    assert torch.cuda.is_available()
    b = SuffixArrayBuilder(0, tune_cache="")
    yield b
    b.close()


def texts():
    rng = np.random.default_rng(77)
    return {
        "repetitive": W.repetitive(copies=40, base_len=5003),       # many later rounds
        "dna": W.dna(1 << 20, seed=0),                              # one later round
        "binary": rng.integers(0, 2, 150001).astype(np.uint8),      # several, shrinking
        "periodic": np.tile(np.frombuffer(b"abcab", np.uint8), 20000),
    }


def build(b, text):
    d = torch.from_numpy(np.ascontiguousarray(text)).to("cuda:0")
    sa = b.build(d)
    torch.cuda.synchronize()
    return sa.cpu().numpy().view(np.uint32), b.last_info()


def test_graph_replays_equal_direct_and_oracle(builder):
    """Each text is built five times in a row with other texts' builds between
    them: the second build captures its later round, the others replay it."""
    T = texts()
    want = {k: oracle.sa(t, parallel=True) for k, t in T.items()}
    builder.set_tuning(round_graphs=1)
    direct = {k: build(builder, t) for k, t in T.items()}
    builder.auto_tuning()
    graph_rounds = 0
    for rep in range(5):
        for k, t in T.items():
            sa, info = build(builder, t)
            assert np.array_equal(sa, want[k]), (k, rep, info)
            assert np.array_equal(sa, direct[k][0])
            assert info["active"] == direct[k][1]["active"], (k, rep)
            assert info["passes_run"] == direct[k][1]["passes_run"]
            if rep >= 2 and info["rounds"] > 1:
                assert info["graph_rounds"] > 0, (k, rep, info)
            graph_rounds += info["graph_rounds"]
            # Eager work of the program itself between replays.
            torch.cuda.synchronize()
            x = torch.arange(1000, device="cuda:0").sum().item()
            assert x == 499500
    assert graph_rounds > 0


@pytest.mark.parametrize("ahead", [1, 2, 3, 16, 64])
@pytest.mark.parametrize("graphs", [0, 1])
def test_rounds_ahead(builder, ahead, graphs):
    """Any number of rounds enqueued per readback gives the same rounds, counts
    and suffix array; rounds past the last one do nothing."""
    builder.set_tuning(rounds_ahead=ahead, round_graphs=graphs)
    try:
        for k, t in texts().items():
            for _ in range(3):
                sa, info = build(builder, t)
            assert np.array_equal(sa, oracle.sa(t, parallel=True)), (k, ahead, graphs)
            assert info["active"][-1] > 0 and len(info["active"]) == info["rounds"], (k, info)
    finally:
        builder.auto_tuning()


def test_round_names_with_rounds_ahead(builder):
    """Stopping after k rounds (sa_build_rounds) caps the rounds run ahead: the
    names equal the closed form for the prefix length reached."""
    t = W.repetitive(copies=12, base_len=3001)
    d = torch.from_numpy(t).to("cuda:0")
    builder.set_tuning(rounds_ahead=8)
    try:
        _, _, full = builder.build_rounds(d, 0)
        for k in range(1, full["rounds"] + 1):
            for _ in range(2):  # the second call replays a captured round
                _, isa, info = builder.build_rounds(d, k)
            assert info["rounds"] == k
            assert np.array_equal(isa.cpu().numpy().view(np.uint32),
                                  oracle.prefix_ranks(t, info["prefix_len"])), (k, info)
    finally:
        builder.auto_tuning()
