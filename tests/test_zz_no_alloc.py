"""rambo_query_seqs_ids_noalloc (the ID-list query with its per-read state
in the library's fixed per-GPU scratch) against rambo_query_seqs_ids, called
through the C ABI: bit-identical id_offsets, IDs and window counts on two
calls in a row, the second with fewer reads (so it runs over what the first
left in the scratch), with both read schedules, on the tiny index and at
the 1024-bit row width; and a batch beyond the scratch is refused on the
host."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import synth
from gpu_util import dev, make_pair, gpu_insert_seqs

pytestmark = pytest.mark.gpu


def with_edges(rd):
    extra = [b"", b"ACGTACG", b"ACGTACGTACGTACGTNACGTACGTACGTACGTACGTAC"]
    parts = [rd.chars] + [np.frombuffer(x, np.uint8) for x in extra]
    off = np.concatenate([rd.offsets, rd.offsets[-1] + np.cumsum([len(x) for x in extra]).astype(np.uint64)])
    return synth.SeqBatch(np.concatenate(parts), off.astype(np.uint64))


def call(g, fn, rd, cap):
    """One raw C-ABI call of fn; (id_offsets, ids, nkmers, status)."""
    L = rb.lib()
    n = rd.n
    off, ch = dev(rd.offsets, np.int64), dev(rd.chars, np.uint8)
    id_off = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
    ids = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    nk = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = getattr(L, fn)(g._h, off.data_ptr(), n, ch.data_ptr(), ch.numel(), id_off.data_ptr(), ids.data_ptr(), cap,
                        nk.data_ptr(), stream)
    assert rc == rb.OK, (fn, rc, L.rambo_last_error(g._h))
    st = L.rambo_sync_status(g._h, stream)
    torch.cuda.synchronize()
    return id_off.cpu().numpy(), ids.cpu().numpy(), nk.cpu().numpy()[:n], st


def check_pair(g, rd, cap):
    a_off, a_ids, a_nk, a_st = call(g, "rambo_query_seqs_ids", rd, cap)
    b_off, b_ids, b_nk, b_st = call(g, "rambo_query_seqs_ids_noalloc", rd, cap)
    assert a_st == b_st == rb.OK
    assert np.array_equal(a_off, b_off)
    assert np.array_equal(a_nk, b_nk)
    total = int(a_off[-1])
    assert np.array_equal(a_ids[:total], b_ids[:total])
    return a_off, a_ids[:total], a_nk


def oracle_ids(o, K, rd):
    m, nk = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    lists = [oracle.mask_to_ids(row, K) for row in m]
    off = np.zeros(len(lists) + 1, np.int64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    return off, np.array([i for x in lists for i in x], np.int64), nk.astype(np.int64)


@pytest.mark.parametrize("mode", [rb.QUERY_WAVE_PER_READ, rb.QUERY_QUEUE])
def test_tiny_two_calls(mode):
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o, g = make_pair(cfg, seed=2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    g.set_query_policy(mode, 512, 8)
    for n, seed in ((3000, 3611), (700, 3612)):   # the second call is smaller
        rd = with_edges(synth.config_batched_reads(sets, n, seed=seed))
        off, ids, nk = check_pair(g, rd, 64 * rd.n)
        w_off, w_ids, w_nk = oracle_ids(o, cfg["K"], rd)
        assert np.array_equal(off, w_off) and np.array_equal(ids, w_ids) and np.array_equal(nk, w_nk)
    g.close()
    o.close()


def test_wide_rows_two_calls_and_limit():
    # the 1024-bit rows of the 100 000-set index (R = 6) with small filters
    cfg = dict(K=4000, B=1000, R=6, eta=2, k=31, m=1 << 14)
    sets = synth.genome_sets(1313, K=cfg["K"], n_ancestors=40, ancestor_len=3000, median_len=800, min_len=200,
                             max_len=3000)
    g = rb.Rambo(**cfg, seed=1314)
    gpu_insert_seqs(g, sets)
    mx = g.noalloc_max_reads()
    per_read = 4 * (cfg["R"] * 1024 // 32 + 5)
    assert 0.9 * rb.NOALLOC_SCRATCH_BYTES / per_read < mx <= rb.NOALLOC_SCRATCH_BYTES / per_read
    for n, seed in ((min(20000, mx), 3621), (1500, 3622)):
        rd = synth.reads(seed, sets, n, median_len=150, min_len=31, max_len=400, substr_frac=0.8,
                         read_sub_rate=0.01)
        off, ids, nk = check_pair(g, rd, int(4 * rd.n) + 1024)
        assert off[-1] > 0
    # more reads than the scratch holds: refused before any work is queued
    L = rb.lib()
    n = mx + 1
    off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")   # n empty reads
    ch = torch.zeros(1, dtype=torch.uint8, device="cuda")
    id_off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = L.rambo_query_seqs_ids_noalloc(g._h, off.data_ptr(), n, ch.data_ptr(), 0, id_off.data_ptr(), None, 0,
                                        None, stream)
    assert rc == rb.EINVAL
    assert b"bytes of scratch" in L.rambo_last_error(g._h)
    assert L.rambo_sync_status(g._h, stream) == rb.OK
    # and the largest batch it holds is taken (all reads empty: empty lists)
    rc = L.rambo_query_seqs_ids_noalloc(g._h, off.data_ptr(), mx, ch.data_ptr(), 0, id_off.data_ptr(), None, 0,
                                        None, stream)
    assert rc == rb.OK and L.rambo_sync_status(g._h, stream) == rb.OK
    assert not id_off[: mx + 1].any().item()
    g.close()
