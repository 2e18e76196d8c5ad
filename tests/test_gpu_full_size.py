"""Parity at the full size of the mid workload (K = 1 000 genome sets, B = 50,
R = 4, m = 2^28, eta = 2; ~2.7e8 inserts), in the launch configuration
bench.py times (rambo_insert_seqs with the automatic policy, batched
rambo_query_kmers).  The oracle builds the whole index on the host; the GPU
index is compared with the oracle's filters bit for bit (every row of every
repetition), through per-cell fill counts, and on sampled queries and
reads."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1910_02611_amd import synth
from gpu_util import dev, host_u32, make_pair, gpu_insert_seqs, first_codes_gpu, first_codes_oracle, gpu_rows

pytestmark = pytest.mark.gpu


def _column_popcounts(g) -> np.ndarray:
    """Number of set bits of every cell (r, b), counted on the GPU over the
    whole bit-sliced index (layout of include/rambo.h)."""
    S = g.row_bits
    assert S >= 32   # one or more whole words per row
    out = np.zeros((g.R, g.B), np.int64)
    for r in range(g.R):
        rows = g.index_words(r * g.words_per_rep, g.m * S // 32).view(g.m, S // 32)
        for b in range(g.B):
            bit = b % 32
            mask = (1 << bit) if bit < 31 else -(1 << 31)   # int32 view of bit 31
            out[r, b] = int(torch.count_nonzero(torch.bitwise_and(rows[:, b // 32], mask)))
        del rows
    return out


@pytest.fixture(scope="module")
def mid():
    cfg = synth.INDEX_MID
    sets = synth.config_mid()
    o, g = make_pair(cfg, seed=2002)
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == 0
    nthreads = min(os.cpu_count() or 1, 16)
    assert o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, nthreads) == 0
    return cfg, sets, o, g, nthreads


def test_mid_fill_counts_every_cell(mid):
    cfg, sets, o, g, _ = mid
    want = o.fill_counts().astype(np.int64)
    assert np.array_equal(_column_popcounts(g), want)
    assert np.array_equal(g.fill_counts().cpu().numpy(), want)   # the library's own counting kernel


def _cell_bytes(rows: torch.Tensor, b: int) -> np.ndarray:
    """Bit b of every row (an [m, S/32] int32 device view of one repetition),
    packed little-endian into m/8 bytes on the device: the layout of one
    oracle filter's words."""
    col = torch.bitwise_and(torch.bitwise_right_shift(rows[:, b // 32], b % 32), 1).to(torch.uint8)
    weights = torch.tensor([1, 2, 4, 8, 16, 32, 64, 128], dtype=torch.uint8, device=rows.device)
    packed = (col.view(-1, 8) * weights).sum(dim=1, dtype=torch.uint8)
    return packed.cpu().numpy()


def test_mid_every_row(mid):
    # the whole index, cell by cell: all m bits of every filter (r, b) equal
    # the oracle's separate filter, and the row padding (bits B..S-1) is zero
    cfg, sets, o, g, _ = mid
    S = g.row_bits
    for r in range(cfg["R"]):
        rows = g.index_words(r * g.words_per_rep, g.m * S // 32).view(g.m, S // 32)
        for b in range(cfg["B"]):
            want = o.bfu_words(r, b).view(np.uint8)
            assert np.array_equal(_cell_bytes(rows, b), want), (r, b)
        pad = torch.zeros_like(rows[:, 0])
        for b in range(cfg["B"], S):
            pad = torch.bitwise_or(pad, torch.bitwise_and(torch.bitwise_right_shift(rows[:, b // 32], b % 32), 1))
        assert int(pad.max()) == 0, r
        del rows


def test_mid_sampled_queries(mid):
    cfg, sets, o, g, nthreads = mid
    q = synth.kmer_queries(3002, sets, 200_000, cfg["k"])   # a prefix-sized sample of the bench's stream
    codes = first_codes_gpu(g, q)
    got = host_u32(g.query_kmers(codes))
    want = o.query_kmers(first_codes_oracle(q, cfg["k"]), nthreads)
    assert np.array_equal(got, want)
    # present queries always report at least one set (zero false negatives)
    assert (got[q.meta["present"]].any(axis=1)).all()


def test_mid_sampled_reads(mid):
    cfg, sets, o, g, nthreads = mid
    rd = synth.reads(3005, sets, 1500, median_len=300, min_len=31, max_len=3000, substr_frac=0.7)
    m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads)
    assert np.array_equal(host_u32(nk), wn.astype(np.uint32))
    assert np.array_equal(host_u32(m), want)
