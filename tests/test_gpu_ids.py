"""Set-ID list answers (rambo_query_seqs_ids) and per-cell fill counts
(rambo_fill_counts) against the oracle, at the tiny workload and at the row
widths of the 10 000- and 100 000-set indexes (with small filters)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import synth
from gpu_util import dev, host_u32, make_pair, gpu_insert_seqs

pytestmark = pytest.mark.gpu


def oracle_ids(o, K, offsets, chars):
    m, nk = o.query_seqs(offsets, chars, nthreads=8)
    lists = [oracle.mask_to_ids(row, K) for row in m]
    off = np.zeros(len(lists) + 1, np.int64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    flat = np.array([i for x in lists for i in x], np.int64)
    return off, flat, nk.astype(np.int64)


def gpu_ids(g, rd, ids=None):
    off, ids, nk = g.query_seqs_ids(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8), ids=ids)
    return off.cpu().numpy(), ids.cpu().numpy().astype(np.int64), nk.cpu().numpy().astype(np.int64)


def check_ids(g, o, K, rd, ids=None):
    w_off, w_ids, w_nk = oracle_ids(o, K, rd.offsets, rd.chars)
    off, got, nk = gpu_ids(g, rd, ids)
    assert np.array_equal(nk, w_nk)
    assert np.array_equal(off, w_off)
    assert np.array_equal(got, w_ids)
    return w_off


def with_edges(rd: synth.SeqBatch) -> synth.SeqBatch:
    """rd plus an empty read, a read shorter than k and one with no valid window."""
    extra = [b"", b"ACGTACG", b"ACGTACGTACGTACGTNACGTACGTACGTACGTACGTAC"]
    parts = [rd.chars] + [np.frombuffer(x, np.uint8) for x in extra]
    lens = [len(x) for x in extra]
    off = np.concatenate([rd.offsets, rd.offsets[-1] + np.cumsum(lens).astype(np.uint64)])
    return synth.SeqBatch(np.concatenate(parts), off.astype(np.uint64))


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o, g = make_pair(cfg, seed=2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    return cfg, sets, o, g


def test_tiny_ids_match_oracle(tiny):
    cfg, sets, o, g = tiny
    rd = with_edges(synth.config_batched_reads(sets, 3000, seed=3011))
    w_off = check_ids(g, o, cfg["K"], rd)
    assert w_off[-1] > 0


def test_ids_overflow_then_retry(tiny):
    cfg, sets, o, g = tiny
    rd = synth.config_batched_reads(sets, 500, seed=3012)
    # capacity 1: the first call overflows (sticky status), the binding calls again
    check_ids(g, o, cfg["K"], rd, ids=torch.empty(1, dtype=torch.int32, device="cuda"))
    assert g.sync_status() == rb.OK


def test_ids_raw_overflow_status(tiny):
    cfg, sets, o, g = tiny
    rd = synth.config_batched_reads(sets, 200, seed=3013)
    n = rd.n
    id_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ids = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    offs, chars = dev(rd.offsets, np.int64), dev(rd.chars, np.uint8)
    rc = rb.lib().rambo_query_seqs_ids(g._h, offs.data_ptr(), n, chars.data_ptr(), chars.numel(),
                                       id_off.data_ptr(), ids.data_ptr(), 4, None, 0)
    assert rc == rb.OK
    assert g.sync_status(torch.cuda.default_stream()) == rb.EOVERFLOW
    w_off, w_ids, _ = oracle_ids(o, cfg["K"], rd.offsets, rd.chars)
    assert np.array_equal(id_off.cpu().numpy(), w_off)
    # only reads whose whole list fits were written
    got = ids.cpu().numpy()
    for q in range(n):
        if w_off[q + 1] <= 4:
            assert np.array_equal(got[w_off[q]:w_off[q + 1]], w_ids[w_off[q]:w_off[q + 1]])
    assert g.sync_status() == rb.OK   # the status was cleared


def test_zero_reads(tiny):
    cfg, sets, o, g = tiny
    off, ids, nk = g.query_seqs_ids(torch.zeros(1, dtype=torch.int64, device="cuda"),
                                    torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert off.cpu().tolist() == [0] and ids.numel() == 0


def test_tiny_fill_counts(tiny):
    cfg, sets, o, g = tiny
    assert np.array_equal(g.fill_counts().cpu().numpy(), o.fill_counts().astype(np.int64))


@pytest.mark.parametrize("K,B,R,m,n_anc,glen", [
    (10_000, 200, 5, 1 << 16, 40, 400),     # row width of the 10 000-set index (S = 256)
    (100_000, 1000, 6, 1 << 14, 100, 160),  # row width of the 100 000-set index (S = 1024)
    (3000, 17, 2, 1 << 12, 6, 300),         # S = 32, odd B
    (50, 3, 7, 1 << 10, 5, 200),            # S = 8, generic repetition count
])
def test_wide_ids_and_fills(K, B, R, m, n_anc, glen):
    cfg = dict(K=K, B=B, R=R, m=m, eta=2, k=31)
    sets = synth.genome_sets(1100 + B, K=K, n_ancestors=n_anc, ancestor_len=glen)
    o, g = make_pair(cfg, seed=2100 + B)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == rb.OK
    assert np.array_equal(g.fill_counts().cpu().numpy(), o.fill_counts().astype(np.int64))
    # 150 bp reads: 80% substrings with 1% further substitutions, 20% random
    rd = with_edges(synth.reads(3100 + B, sets, 1500, median_len=150, min_len=150, max_len=150,
                                substr_frac=0.8, read_sub_rate=0.01))
    check_ids(g, o, K, rd)
    m_gpu, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    want, _ = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    assert np.array_equal(host_u32(m_gpu), want)


@pytest.fixture(scope="module")
def wide_long():
    """1 024-bit rows (B = 1 000, R = 6) over set genomes of about 1.5 kbp, so
    reads span several 256-window blocks of the read probing."""
    cfg = dict(K=20_000, B=1000, R=6, m=1 << 14, eta=2, k=31)
    sets = synth.genome_sets(1177, K=cfg["K"], n_ancestors=60, ancestor_len=1500)
    o, g = make_pair(cfg, seed=2177)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == rb.OK
    return cfg, sets, o, g


def long_reads(sets, seed):
    """Reads of 31..1 400 bp (85% substrings with a few substitutions), every
    7th in lower case and every 11th with an N, plus the edge reads."""
    rd = synth.reads(seed, sets, 600, median_len=400, min_len=31, max_len=1400, substr_frac=0.85,
                     read_sub_rate=0.002)
    chars = rd.chars.copy()
    rng = np.random.default_rng(seed)
    for q in range(rd.n):
        a, b = int(rd.offsets[q]), int(rd.offsets[q + 1])
        if q % 7 == 0:
            chars[a:b] = np.char.lower(chars[a:b].view("S1")).view(np.uint8)
        if q % 11 == 0 and b > a:
            chars[a + int(rng.integers(0, b - a))] = ord("N")
    return with_edges(synth.SeqBatch(chars, rd.offsets))


@pytest.fixture(scope="module")
def long_batch(wide_long):
    """The long-read batch and the oracle's answers to it (computed once)."""
    cfg, sets, o, g = wide_long
    rd = long_reads(sets, 3177)
    want, w_nk = o.query_seqs(rd.offsets, rd.chars, nthreads=16)
    lists = [oracle.mask_to_ids(row, cfg["K"]) for row in want]
    w_off = np.zeros(len(lists) + 1, np.int64)
    np.cumsum([len(x) for x in lists], out=w_off[1:])
    w_ids = np.array([i for x in lists for i in x], np.int64)
    return rd, want, w_nk.astype(np.int64), w_off, w_ids


@pytest.mark.parametrize("mode,chunk", [(rb.QUERY_WAVE_PER_READ, 0), (rb.QUERY_QUEUE, 256), (rb.QUERY_QUEUE, 1024)])
def test_multi_block_reads_match_oracle(wide_long, long_batch, mode, chunk):
    """The read probing takes repetition 0 over a block of windows (after a
    first look at a few spread over it) before the other repetitions: answers
    and ID lists for reads of one to six blocks, split or not into queue
    chunks, equal the oracle's term-by-term ones."""
    cfg, sets, o, g = wide_long
    rd, want, w_nk, w_off, w_ids = long_batch
    g.set_query_policy(mode, chunk, 8 if chunk else 0)
    try:
        off, got, nk = gpu_ids(g, rd)
        assert np.array_equal(nk, w_nk)
        assert np.array_equal(off, w_off)
        assert np.array_equal(got, w_ids)
        m_gpu, nk2 = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
        assert np.array_equal(host_u32(m_gpu), want)
        assert np.array_equal(nk2.cpu().numpy().astype(np.int64), w_nk)
    finally:
        g.set_query_policy()
    # the batch holds both kinds of reads
    sizes = np.diff(w_off)
    assert (sizes > 0).sum() > 50 and (sizes == 0).sum() > 50


def test_ids_without_waiting(tiny):
    """wait=False: one asynchronous call into the caller's buffers; after the
    stream is done the lists equal the synchronous form's, and a capacity
    that is too small shows as EOVERFLOW (the offsets stay complete)."""
    cfg, sets, o, g = tiny
    rd = synth.config_batched_reads(sets, 800, seed=3014)
    offs, chars = dev(rd.offsets, np.int64), dev(rd.chars, np.uint8)
    w_off, w_ids, w_nk = g.query_seqs_ids(offs, chars)
    id_off = torch.empty(rd.n + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(int(w_off[-1].item()) + 16, dtype=torch.int32, device="cuda")
    off, got, nk = g.query_seqs_ids(offs, chars, ids=ids, id_offsets=id_off, wait=False)
    assert g.sync_status() == rb.OK
    assert torch.equal(off, w_off) and torch.equal(nk[:rd.n], w_nk)
    assert torch.equal(got[:int(off[-1].item())], w_ids)
    small = torch.empty(max(1, int(w_off[-1].item()) // 2), dtype=torch.int32, device="cuda")
    off2, _, _ = g.query_seqs_ids(offs, chars, ids=small, id_offsets=id_off, wait=False)
    assert g.sync_status() == rb.EOVERFLOW
    assert torch.equal(off2, w_off)
    assert g.sync_status() == rb.OK
