"""Tuning cache: the host-only lookup in a JSON cache file (no GPU), and on the
GPU the autotuner's search, its saved table, and builds that pick the table's
entry up. Tuning never changes a result, so the GPU test also checks the
arrays against the oracle."""

import json
import os

import numpy as np
import pytest

from paper_1610_03007_amd import SAError, _native

FORMAT = "sa_mi355x_tune/1"


def entry(**kw):
    e = {"arch": "gfx950", "mode": "single", "log2n": 28, "code_bits": 7, "sort_items": 16,
         "sort_wgs_per_cu": 2, "lazy_ratio": 8, "round0_full": 0, "ms": 20.0}
    e.update(kw)
    return e


def write(tmp_path, entries, fmt=FORMAT):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"format": fmt, "entries": entries}))
    return str(p)


def test_tuning_struct_layout():
    """The binding's sa_tuning mirror has the header's eleven 32-bit fields, in
    order (the library writes the whole struct)."""
    import ctypes
    names = [f[0] for f in _native.Tuning._fields_]
    assert names == ["sort_items", "lazy_ratio", "round0_full", "sort_wgs_per_cu", "sort_block",
                     "sort_match", "radix_bits", "rounds_ahead", "round_graphs", "prefix_mult",
                     "isa_direct"]
    assert ctypes.sizeof(_native.Tuning) == 44
    header = open(os.path.join(os.path.dirname(__file__), "..", "include", "sa.h")).read()
    body = header[header.index("typedef struct {\n  uint32_t sort_items;"):]
    body = body[:body.index("} sa_tuning;")]
    fields = [line.split()[1].rstrip(";").split("[")[0] for line in body.splitlines()[1:]
              if line.strip().startswith("uint32_t")]
    assert fields == names


def test_missing_file_gives_defaults(tmp_path):
    found, t = _native.tune_lookup(str(tmp_path / "none.json"), "gfx950", "single", 1 << 20)
    assert not found
    assert t["sort_items"] in (8, 12, 16, 20, 24) and t["lazy_ratio"] >= 3


def test_nearest_size_bucket(tmp_path):
    p = write(tmp_path, [entry(log2n=20, sort_items=8), entry(log2n=28, sort_items=24),
                         entry(log2n=30, sort_items=12)])
    assert _native.tune_lookup(p, "gfx950", "single", 1 << 20)[1]["sort_items"] == 8
    assert _native.tune_lookup(p, "gfx950", "single", (1 << 21) + 5)[1]["sort_items"] == 8
    assert _native.tune_lookup(p, "gfx950", "single", 1 << 28)[1]["sort_items"] == 24
    assert _native.tune_lookup(p, "gfx950", "single", (1 << 29) + 1)[1]["sort_items"] == 24
    assert _native.tune_lookup(p, "gfx950", "single", 1 << 31)[1]["sort_items"] == 12
    # More than two binary orders of magnitude from every entry: defaults.
    assert not _native.tune_lookup(p, "gfx950", "single", 1 << 24)[0]
    assert not _native.tune_lookup(p, "gfx950", "single", 1000)[0]


def test_arch_mode_and_code_width(tmp_path):
    p = write(tmp_path, [entry(code_bits=3, sort_items=8), entry(code_bits=7, sort_items=20),
                         entry(mode="batch", code_bits=0, sort_items=12)])
    n = 1 << 28
    assert not _native.tune_lookup(p, "gfx942", "single", n)[0]
    assert _native.tune_lookup(p, "gfx950", "single", n, 3)[1]["sort_items"] == 8
    assert _native.tune_lookup(p, "gfx950", "single", n, 2)[1]["sort_items"] == 8
    assert _native.tune_lookup(p, "gfx950", "single", n, 7)[1]["sort_items"] == 20
    assert _native.tune_lookup(p, "gfx950", "single", n, 8)[1]["sort_items"] == 20
    found, t = _native.tune_lookup(p, "gfx950", "batch", n, 5)
    assert found and t["sort_items"] == 12
    with pytest.raises(SAError):
        _native.tune_lookup(p, "gfx950", "serve", n)


def test_knobs_round_trip(tmp_path):
    p = write(tmp_path, [entry(sort_items=12, sort_wgs_per_cu=6, lazy_ratio=64, round0_full=1)])
    found, t = _native.tune_lookup(p, "gfx950", "single", 1 << 28, 7)
    assert found
    assert t == {"sort_items": 12, "sort_wgs_per_cu": 6, "lazy_ratio": 64, "round0_full": 1,
                 "sort_block": 256, "sort_match": 0, "radix_bits": 8, "rounds_ahead": 0,
                 "round_graphs": 0, "prefix_mult": 2, "isa_direct": 0}
    p = write(tmp_path, [entry(sort_items=8, sort_block=512, sort_match=1)])
    t = _native.tune_lookup(p, "gfx950", "single", 1 << 28, 7)[1]
    assert t["sort_block"] == 512 and t["sort_match"] == 1


@pytest.mark.parametrize("bad", [
    "{", "[]", '{"format": "other/1", "entries": []}', '{"format": "%s"}' % FORMAT,
    '{"format": "%s", "entries": [{"arch": "gfx950"}]}' % FORMAT,
    '{"format": "%s", "entries": []} trailing' % FORMAT,
])
def test_malformed_files_are_rejected(tmp_path, bad):
    p = tmp_path / "bad.json"
    p.write_text(bad)
    with pytest.raises(SAError):
        _native.tune_lookup(str(p), "gfx950", "single", 1 << 20)


@pytest.mark.parametrize("knob", [{"sort_items": 10}, {"lazy_ratio": 2}, {"round0_full": 2},
                                  {"sort_wgs_per_cu": 17}, {"log2n": 64}, {"mode": "serve"},
                                  {"sort_block": 384}, {"sort_block": 512, "sort_items": 16},
                                  {"sort_items": 4}, {"sort_match": 2},
                                  {"radix_bits": 5}, {"radix_bits": 10},
                                  {"radix_bits": 7, "sort_block": 256, "sort_items": 8},
                                  {"radix_bits": 6, "sort_block": 512, "sort_items": 8,
                                   "sort_match": 1},
                                  {"radix_bits": 9, "sort_block": 512, "sort_items": 12},
                                  {"radix_bits": 9, "sort_block": 512, "sort_items": 4}])
def test_invalid_knobs_are_rejected(tmp_path, knob):
    p = write(tmp_path, [entry(**knob)])
    with pytest.raises(SAError):
        _native.tune_lookup(p, "gfx950", "single", 1 << 28)


@pytest.mark.gpu
def test_autotune_save_and_reuse(tmp_path):
    import torch

    import oracle
    import workloads as W
    from paper_1610_03007_amd import SuffixArrayBuilder

    n = 1 << 18
    text = W.dna(n, seed=77)
    d = torch.from_numpy(text).to("cuda:0")
    path = str(tmp_path / "tune.json")
    b = SuffixArrayBuilder(0, tune_cache=path)
    try:
        best, ms = b.tune(d, reps=1)
        assert ms > 0
        assert best["sort_items"] in (4, 8, 12, 16, 20, 24) and best["sort_block"] in (256, 512)
        b.save_tuning()
        doc = json.load(open(path))
        assert doc["format"] == FORMAT and len(doc["entries"]) == 1
        e = doc["entries"][0]
        assert e["mode"] == "single" and e["log2n"] == 18 and e["code_bits"] == 3
        # The cache holds the searched knobs; the launch policies are not tuned.
        searched = {k: v for k, v in best.items()
                    if k not in ("rounds_ahead", "round_graphs", "isa_direct")}
        assert {k: e[k] for k in searched} == searched
        # The tuner leaves automatic choice in force: the next build uses the entry.
        sa = b.build(d, sigma=4)
        torch.cuda.synchronize()
        assert b.tuning_source() == "cache" and b.tuning() == best
        assert np.array_equal(sa.cpu().numpy().view(np.uint32), oracle.sa(text))
    finally:
        b.close()
    # A fresh context reads the file; an explicit tuning wins until dropped.
    b2 = SuffixArrayBuilder(0, tune_cache=path)
    try:
        other = 8 if best["sort_items"] != 8 else 12
        b2.set_tuning(sort_items=other, sort_block=512, radix_bits=8)
        sa = b2.build(d)
        torch.cuda.synchronize()
        assert b2.tuning_source() == "explicit" and b2.tuning()["sort_items"] == other
        assert np.array_equal(sa.cpu().numpy().view(np.uint32), oracle.sa(text))
        b2.auto_tuning()
        b2.build(d)
        torch.cuda.synchronize()
        assert b2.tuning_source() == "cache" and b2.tuning() == best
        # Far from every entry: the defaults.
        small = torch.from_numpy(W.dna(1 << 12, seed=5)).to("cuda:0")
        b2.build(small)
        torch.cuda.synchronize()
        assert b2.tuning_source() == "default"
    finally:
        b2.close()


@pytest.mark.gpu
def test_autotune_batch_mode(tmp_path):
    import torch

    import oracle
    import workloads as W
    from paper_1610_03007_amd import SuffixArrayBuilder

    texts = [W.dna(3000 + 17 * i, seed=i) for i in range(40)]
    off = np.zeros(len(texts) + 1, np.uint64)
    np.cumsum([t.size for t in texts], out=off[1:])
    d = torch.from_numpy(np.concatenate(texts)).to("cuda:0")
    path = str(tmp_path / "tune.json")
    b = SuffixArrayBuilder(0, tune_cache=path)
    try:
        best, ms = b.tune(d, off, reps=1)
        b.save_tuning()
        e = json.load(open(path))["entries"][0]
        assert e["mode"] == "batch" and e["code_bits"] == 0
        sa = b.build_batch(d, off).cpu().numpy().view(np.uint32)
        assert b.tuning_source() == "cache" and b.tuning() == best
        for t, text in enumerate(texts):
            assert np.array_equal(sa[int(off[t]):int(off[t + 1])], oracle.sa(text))
    finally:
        b.close()


@pytest.mark.parametrize("rb,items", [(6, 4), (6, 12), (7, 8), (9, 8), (8, 12)])
def test_digit_width_entries(tmp_path, rb, items):
    """Entries carry the radix digit width; widths other than 8 bits take
    512-thread sweeps of 4, 8 or 12 items (8 at 9 bits)."""
    p = write(tmp_path, [entry(radix_bits=rb, sort_block=512, sort_items=items)])
    found, t = _native.tune_lookup(p, "gfx950", "single", 1 << 28, 7)
    assert found and t["radix_bits"] == rb and t["sort_items"] == items
