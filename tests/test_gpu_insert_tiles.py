"""Tile shapes of the partitioned insert (rambo_set_insert_tiles): every
shape gives the oracle's index bits (Alg. 1), from sequences (piece stage A)
and from codes; out-of-range shapes are refused on the host."""
import numpy as np
import pytest

from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import synth
from gpu_util import dev, host_u32, make_pair

pytestmark = pytest.mark.gpu

# 4 x 2^22 rows of 64 bits: 2^30 index bits, 8 coarse buckets by default
CFG = dict(K=300, B=50, R=4, eta=2, k=31, m=1 << 22)


@pytest.fixture(scope="module")
def pair():
    sets = synth.genome_sets(4401, K=CFG["K"], n_ancestors=12, ancestor_len=60000, median_len=20000, min_len=2000,
                             max_len=60000)
    o, g = make_pair(CFG, seed=4402)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    want = np.concatenate([np.stack([o.bfu_bits(r, b) for b in range(CFG["B"])], axis=1)
                           for r in range(CFG["R"])])   # [R*m, B]
    g.set_insert_policy(rb.INSERT_PARTITIONED)
    return sets, g, want


def index_bits(g):
    words = host_u32(g.index_words()).reshape(CFG["R"] * CFG["m"], -1)
    bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :CFG["B"]], bits[:, CFG["B"]:]


@pytest.mark.parametrize("tiles", [
    dict(),
    dict(steps=1),
    dict(steps=2, stage_b_tile=8192),
    dict(stage_b_tile=16384, groups=2),
    dict(stage_b_tile=32768, groups=8, fine_bits=9),
    dict(steps=1, groups=4, fine_bits=12),
    dict(fine_bits=10, groups=1),
])
def test_tiles_give_the_oracle_index(pair, tiles):
    sets, g, want = pair
    g.set_insert_tiles(**tiles)
    g.clear()
    g.insert_seqs(dev(sets.set_ids, np.int32), dev(sets.offsets, np.int64), dev(sets.chars, np.uint8))
    assert g.sync_status() == rb.OK
    eff = g.insert_tiles()
    na = max(1, (1 << 30) >> (20 + eff["fine_bits"]))   # coarse buckets (regions of 2^20 bits)
    for k, v in tiles.items():
        assert eff[k] == (min(v, na) if k == "groups" else v), (k, eff)
    got, pad = index_bits(g)
    assert np.array_equal(got, want)
    assert not pad.any()
    g.set_insert_tiles()


def test_tiles_from_codes(pair):
    sets, g, want = pair
    codes = g.extract_kmers(dev(sets.offsets, np.int64), dev(sets.chars, np.uint8))
    g.set_insert_tiles(stage_b_tile=32768, groups=2, fine_bits=11)
    g.clear()
    # every window's code (invalid ones are skipped by the code path too)
    valid = codes != -1
    import torch
    idx = torch.nonzero(valid).flatten()
    seq = torch.searchsorted(torch.from_numpy(sets.offsets[1:].astype(np.int64)).cuda(), idx, right=True)
    counts = torch.bincount(seq, minlength=sets.n)
    off = torch.zeros(sets.n + 1, dtype=torch.int64, device="cuda")
    off[1:] = torch.cumsum(counts, 0)
    g.insert_kmers(dev(sets.set_ids, np.int32), off, codes[idx].contiguous())
    assert g.sync_status() == rb.OK
    got, _ = index_bits(g)
    assert np.array_equal(got, want)
    g.set_insert_tiles()


def test_bad_tiles_are_refused(pair):
    _, g, _ = pair
    for bad in (dict(steps=3), dict(stage_b_tile=4096), dict(groups=3), dict(fine_bits=7), dict(fine_bits=13)):
        with pytest.raises(rb.RamboError):
            g.set_insert_tiles(**bad)
    assert g.insert_tiles()["fine_bits"] == 8


def test_insert_autotuner_keeps_the_index(pair, tmp_path, monkeypatch):
    # the tuner's sweep checks every shape against the first one; its pick,
    # applied to the handle, still gives the oracle's index
    sets, g, want = pair
    from paper_1910_02611_amd import autotune
    monkeypatch.setenv("RAMBO_TUNE_CACHE", str(tmp_path / "tune.json"))
    d = (dev(sets.set_ids, np.int32), dev(sets.offsets, np.int64), dev(sets.chars, np.uint8))
    r = autotune.tune_insert(g, lambda: g.insert_seqs(*d), "tiles-test", reps=1)
    assert not r["cached"] and len(r["sweep"]) >= 4
    assert r["seconds"] <= r["automatic_seconds"]
    g.clear()
    g.insert_seqs(*d)
    got, _ = index_bits(g)
    assert np.array_equal(got, want)
    again = autotune.tune_insert(g, lambda: g.insert_seqs(*d), "tiles-test", reps=1)
    assert again["cached"] and again["tiles"] == r["tiles"]
    g.set_insert_tiles()
