"""The work-queue launch of batched sequence queries gives the oracle's answers
for every tile shape, including chunks far smaller than the reads (many
chunks per read, early exit across chunks) and grids smaller than the work."""
import numpy as np
import pytest

from paper_1910_02611_amd import synth
from paper_1910_02611_amd import rambo as rb
import oracle
from gpu_util import dev, host_u32, make_pair, gpu_insert_seqs, gpu_index_bits, oracle_index_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o, g = make_pair(cfg, seed=2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    rd = synth.config_batched_reads(sets, 2500, seed=3009)
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    return cfg, sets, g, rd, want, wn.astype(np.uint32)


@pytest.mark.parametrize("mode,chunk,wpc", [
    (rb.QUERY_WAVE_PER_READ, 0, 0),
    (rb.QUERY_QUEUE, 0, 0),
    (rb.QUERY_QUEUE, 64, 1),
    (rb.QUERY_QUEUE, 100, 2),
    (rb.QUERY_QUEUE, 4096, 32),
    (rb.QUERY_QUEUE, 1 << 20, 4),
])
def test_queue_tiles_match_oracle(tiny, mode, chunk, wpc):
    cfg, sets, g, rd, want, wn = tiny
    g.set_query_policy(mode, chunk, wpc)
    try:
        for _ in range(2):   # the per-read state is reset by every call
            m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
            assert np.array_equal(host_u32(nk), wn)
            assert np.array_equal(host_u32(m), want)
    finally:
        g.set_query_policy(rb.QUERY_AUTO)


def test_queue_grows_its_state(tiny):
    cfg, sets, g, rd, want, wn = tiny
    # a first small batch, then the full one: the state is regrown in place
    few = synth.SeqBatch(rd.chars[: int(rd.offsets[10])].copy(), rd.offsets[:11].copy())
    m, _ = g.query_seqs(dev(few.offsets, np.int64), dev(few.chars, np.uint8))
    assert np.array_equal(host_u32(m), want[:10])
    m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    assert np.array_equal(host_u32(m), want) and np.array_equal(host_u32(nk), wn)


def test_queue_mid_shape_reads():
    """Another row width and shape (B = 50: two-word rows; R = 4)."""
    cfg = dict(K=200, B=50, R=4, eta=2, k=31, m=1 << 16)
    sets = synth.genome_sets(4242, K=200, n_ancestors=10, ancestor_len=3000)
    o, g = make_pair(cfg, seed=77)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    rd = synth.reads(4243, sets, 800, median_len=400, min_len=1, max_len=3000, substr_frac=0.8)
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    for chunk in (0, 128):
        g.set_query_policy(rb.QUERY_QUEUE, chunk, 0)
        m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
        assert np.array_equal(host_u32(nk), wn.astype(np.uint32))
        assert np.array_equal(host_u32(m), want)


@pytest.mark.parametrize("mode", [rb.QUERY_WAVE_PER_READ, rb.QUERY_QUEUE])
def test_captured_graph_replays_match_oracle(tiny, mode):
    # the batched query recorded once as a graph and replayed several times,
    # with eager calls (other inputs) in between: every replay gives the
    # oracle's answers
    from paper_1910_02611_amd import autotune
    import torch
    cfg, sets, g, rd, want, wn = tiny
    g.set_query_policy(mode, 256, 8)
    try:
        off, ch = dev(rd.offsets, np.int64), dev(rd.chars, np.uint8)
        out = torch.empty((rd.n, g.W), dtype=torch.int32, device="cuda")
        nk = torch.empty(rd.n, dtype=torch.int32, device="cuda")
        graph = autotune.capture_query_seqs(g, off, ch, out, nk)
        other = synth.config_batched_reads(sets, 300, seed=3019)
        for _ in range(3):
            out.zero_()
            nk.zero_()
            graph.replay()
            g.query_seqs(dev(other.offsets, np.int64), dev(other.chars, np.uint8))   # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(host_u32(nk), wn)
            assert np.array_equal(host_u32(out), want)
    finally:
        g.set_query_policy(rb.QUERY_AUTO)


@pytest.mark.parametrize("policy", [rb.INSERT_PARTITIONED, rb.INSERT_DIRECT])
def test_captured_insert_pipelines_match_oracle(policy):
    # a recorded [clear + insert A] and a recorded [insert B], replayed in
    # several orders with eager work between the replays: every state equals
    # the oracle's (a recorded insert reads its regions back, so it never
    # drops bits that another insert put there)
    import torch
    from paper_1910_02611_amd import autotune
    cfg = dict(K=100, B=50, R=4, eta=2, k=31, m=1 << 14)
    sets = synth.genome_sets(4301, K=100, n_ancestors=5, ancestor_len=600, sub_rate=0.02)
    half = sets.n // 2
    A = synth.SeqBatch(sets.chars, sets.offsets[: half + 1], sets.set_ids[:half])
    Bs = synth.SeqBatch(sets.chars, sets.offsets[half:], sets.set_ids[half:])
    oa = oracle.OracleIndex(**cfg, seed=31)
    oa.insert_seqs(A.set_ids, A.offsets, A.chars, 8)
    oab = oracle.OracleIndex(**cfg, seed=31)
    oab.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    ob = oracle.OracleIndex(**cfg, seed=31)
    ob.insert_seqs(Bs.set_ids, Bs.offsets, Bs.chars, 8)
    g = rb.Rambo(**cfg, seed=31)
    g.set_insert_policy(policy, 1 << 20)    # small scratch: several batches per insert
    dA = (dev(A.set_ids, np.int32), dev(A.offsets, np.int64), dev(A.chars, np.uint8))
    dB = (dev(Bs.set_ids, np.int32), dev(Bs.offsets, np.int64), dev(Bs.chars, np.uint8))
    g_clear_a = autotune.capture(lambda: (g.clear(), g.insert_seqs(*dA)))
    g_b = autotune.capture(lambda: g.insert_seqs(*dB))
    q = synth.kmer_queries(4302, sets, 2000, 31)
    codes = dev(oracle.extract(q.offsets, q.chars, 31)[q.offsets[:-1].astype(np.int64)], np.int64)
    for _ in range(3):
        g_clear_a.replay()
        torch.cuda.synchronize()
        assert np.array_equal(gpu_index_bits(g), oracle_index_bits(oa))
        g_b.replay()
        g.query_kmers(codes)                       # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(gpu_index_bits(g), oracle_index_bits(oab))
        g.clear()                                  # eager: the index is known to be zero
        g_b.replay()
        torch.cuda.synchronize()
        assert np.array_equal(gpu_index_bits(g), oracle_index_bits(ob))
        g.insert_seqs(*dA)                         # eager insert after the replay
        torch.cuda.synchronize()
        assert np.array_equal(gpu_index_bits(g), oracle_index_bits(oab))
    assert g.sync_status() == rb.OK
    g.close()
