"""GPU tests of the continuous-batching server: every request's suffix array
equals the oracle's and the array the same text gets alone, whatever else is in
flight (bit-exact)."""

import threading
import time

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def texts_mix(seed, count, max_len):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice([1, 2, 5, int(rng.integers(6, max_len))]))
        k = i % 5
        if k == 0:
            t = W.dna(n, seed=int(rng.integers(1 << 30)))
        elif k == 1:
            t = W.markov3(n, chain_seed=int(rng.integers(1 << 30)))
        elif k == 2:
            t = rng.integers(0, 2, n).astype(np.uint8)
        elif k == 3:
            t = np.full(n, 97, np.uint8)
        else:
            t = W.repetitive(copies=8, base_len=max(1, n // 8))[:n]
        out.append(np.ascontiguousarray(t, dtype=np.uint8))
    return out


def drain(srv, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            done, sa, lat = srv.poll(t)
            if done:
                res[t] = (sa, lat)
        if time.time() - t0 > timeout:
            raise AssertionError(f"server did not finish: {len(res)}/{len(tickets)} done, "
                                 f"{srv.stats()}")
        time.sleep(0.001)
    return res


@pytest.fixture(scope="module")
def server():
    from paper_1610_03007_amd import SuffixArrayServer
    assert torch.cuda.is_available()
    srv = SuffixArrayServer(0, capacity_bytes=4 << 30, max_text=1 << 22)
    yield srv
    srv.close()


@pytest.fixture(scope="module")
def builder():
    from paper_1610_03007_amd import SuffixArrayBuilder
    b = SuffixArrayBuilder(0)
    yield b
    b.close()


def test_server_matches_oracle_and_alone(server, builder):
    texts = texts_mix(1, 80, 200000)
    tickets = [server.submit(t) for t in texts]
    res = drain(server, tickets)
    for t, text in zip(tickets, texts):
        sa, lat = res[t]
        assert lat is not None and lat >= 0
        want = oracle.sa(text)
        assert np.array_equal(sa, want), (text.size,)
        alone = builder.build(torch.from_numpy(text.copy()).to("cuda:0"))
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy().view(np.uint32), sa)


def test_server_arrivals_while_running(server):
    """Requests arrive while earlier ones are on the GPU and join later rounds."""
    texts = texts_mix(2, 120, 400000)
    tickets = [None] * len(texts)
    rng = np.random.default_rng(3)

    def producer():
        for i, t in enumerate(texts):
            tickets[i] = server.submit(t)
            time.sleep(float(rng.exponential(0.002)))

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    res = drain(server, tickets)
    for t, text in zip(tickets, texts):
        assert np.array_equal(res[t][0], oracle.sa(text))
    st = server.stats()
    assert st["failed"] == 0


def test_server_admission_by_footprint():
    """A small device budget admits only a few texts at a time; the rest wait
    and are admitted as earlier ones finish."""
    from paper_1610_03007_amd import SAError, SuffixArrayServer
    srv = SuffixArrayServer(0, capacity_bytes=50 * 1_200_000, max_text=1 << 20)
    try:
        texts = [W.markov3(500000, chain_seed=s) for s in range(8)] + \
                [W.dna(300000, seed=s) for s in range(4)]
        tickets = [srv.submit(t) for t in texts]
        assert srv.stats()["arena_positions"] < 2 * 500000 + 300000
        res = drain(srv, tickets)
        for t, text in zip(tickets, texts):
            assert np.array_equal(res[t][0], oracle.sa(text))
        with pytest.raises(SAError):
            srv.submit(np.zeros((1 << 20) + 1, np.uint8))  # above max_text
    finally:
        srv.close()


def test_server_empty_and_tiny(server):
    tickets = [server.submit(b""), server.submit(b"x"), server.submit(b"banana")]
    res = drain(server, tickets)
    assert res[tickets[0]][0].tolist() == []
    assert res[tickets[1]][0].tolist() == [0]
    assert res[tickets[2]][0].tolist() == [5, 3, 1, 0, 4, 2]


def test_server_concurrent_clients(server):
    """Several host threads submit and poll at once; every result is exact."""
    texts = texts_mix(7, 96, 150000)
    results = {}
    errors = []

    def client(k):
        try:
            mine = texts[k::4]
            tickets = [server.submit(t) for t in mine]
            got = drain(server, tickets)
            for t, text in zip(tickets, mine):
                results[(k, t)] = (got[t][0], text)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    assert len(results) == len(texts)
    for sa, text in results.values():
        assert np.array_equal(sa, oracle.sa(text))


def test_server_poll_into_device_tensor(server):
    """poll() fills a caller's device tensor instead of host memory."""
    text = W.markov3(300001, chain_seed=44)
    t = server.submit(text)
    out = torch.empty(text.size, dtype=torch.int32, device="cuda:0")
    t0 = time.time()
    while True:
        done, sa, lat = server.poll(t, out=out)
        if done:
            break
        assert time.time() - t0 < 120
        time.sleep(0.001)
    assert sa is out
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.sa(text))


def test_server_max_text_boundary():
    """A text of exactly max_text bytes is accepted; one byte more is refused."""
    from paper_1610_03007_amd import SAError, SuffixArrayServer
    max_text = 1 << 18
    srv = SuffixArrayServer(0, capacity_bytes=64 << 20, max_text=max_text)
    try:
        text = W.dna(max_text, seed=8)
        t = srv.submit(text)
        res = drain(srv, [t])
        assert np.array_equal(res[t][0], oracle.sa(text))
        with pytest.raises(SAError):
            srv.submit(np.zeros(max_text + 1, np.uint8))
        st = srv.stats()
        assert st["completed"] >= 1 and st["failed"] == 0
    finally:
        srv.close()
