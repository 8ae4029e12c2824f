"""Input generators: deterministic, right shapes and alphabets (no GPU)."""

import numpy as np

import workloads as W


def test_dna():
    a = W.dna(1 << 16, 0)
    assert a.dtype == np.uint8 and a.size == 1 << 16
    assert set(np.unique(a).tolist()) == set(b"ACGT")
    assert np.array_equal(a, W.dna(1 << 16, 0))
    assert not np.array_equal(a, W.dna(1 << 16, 1))


def test_markov():
    m = W.markov3(100000, chain_seed=2)
    assert m.size == 100000
    assert set(np.unique(m).tolist()) <= set(W.SYMBOLS96.tolist())
    assert np.array_equal(m, W.markov3(100000, chain_seed=2))
    # segmented generation keeps the prefix of a longer text deterministic
    big = W.markov3(W.MARKOV_SEGMENT + 1000, chain_seed=2)
    assert big.size == W.MARKOV_SEGMENT + 1000
    assert np.array_equal(big, W.markov3(W.MARKOV_SEGMENT + 1000, chain_seed=2))


def test_markov_table_rows_are_cumulative():
    tab = W.markov_table(1)
    assert tab.shape == (96 ** 3, 95)
    rows = tab[:1000].astype(np.int64)
    assert (np.diff(rows, axis=1) >= 0).all()


def test_repetitive():
    r = W.repetitive(copies=16, base_len=4096)
    assert r.size == 16 * 4096
    copies = r.reshape(16, 4096)
    diff = (copies != copies[0]).sum()
    assert 0 < diff < 50  # about 2 * 16 * 4096 * 1e-4 differing positions
    assert np.array_equal(r, W.repetitive(copies=16, base_len=4096))


def test_batch():
    texts, off = W.batch(num_texts=8, lo=100, hi=1000)
    assert off.dtype == np.uint64 and off.size == 9 and int(off[-1]) == texts.size
    lens = np.diff(off.astype(np.int64))
    assert (lens >= 100).all() and (lens < 1000).all()
    assert set(np.unique(texts[off[0]:off[1]]).tolist()) <= set(b"ACGT")
