"""GPU parity of the raw 64-bit key path (documents as sets, word unigrams as
terms, Sec. 5.3): with RAMBO_FLAG_RAW_KEYS the device index and the answers
of word queries equal the oracle's raw-key index bit for bit, on seeded
synthetic documents (a Zipf vocabulary of random 64-bit word keys), up to the
full size of the Wikipedia-sample index (K = 17 618, B = 2 000, R = 2,
m = 200 000)."""
import numpy as np
import pytest

import oracle
from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import synth
from gpu_util import dev, host_u32, gpu_index_bits, oracle_index_bits, gpu_rows

pytestmark = pytest.mark.gpu


def _pair(cfg, seed):
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed, oracle.FLAG_RAW_KEYS)
    g = rb.Rambo(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed, rb.FLAG_RAW_KEYS)
    return o, g


def _insert(o, g, docs):
    assert o.insert_kmers(docs.set_ids, docs.offsets, docs.keys, 8) == 0
    g.insert_kmers(dev(docs.set_ids, np.int32), dev(docs.offsets, np.int64), dev(docs.keys, np.int64))
    assert g.sync_status() == rb.OK


SHAPES = [
    dict(K=40, B=8, R=3, eta=2, k=31, m=3000),        # S = 8: four rows per word
    dict(K=200, B=50, R=2, eta=4, k=5, m=1 << 13),    # keys far beyond 4^k
    dict(K=600, B=200, R=4, eta=3, k=31, m=5000),
    dict(K=3000, B=2000, R=2, eta=4, k=31, m=4096),   # 2048-bit rows
    dict(K=4096, B=1000, R=2, eta=3, k=31, m=4096),   # answers of 128 words (16-byte stores)
]


@pytest.mark.parametrize("cfg", SHAPES, ids=lambda c: "K%(K)d-B%(B)d-R%(R)d-e%(eta)d-m%(m)d" % c)
def test_documents_match_oracle(cfg):
    seed = cfg["B"] + 11
    docs = synth.documents(seed, cfg["K"], vocab=20_000, median_len=80, min_len=1, max_len=600)
    o, g = _pair(cfg, seed)
    _insert(o, g, docs)
    assert np.array_equal(g.partition(), o.phi())
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    q = synth.word_queries(seed + 1, docs, 5000)
    want = o.query_kmers(q, nthreads=8)
    got = host_u32(g.query_kmers(dev(q, np.int64)))
    assert np.array_equal(got, want)
    assert np.array_equal(host_u32(g.query_kmers(dev(q[:300], np.int64), plain=True)), want[:300])
    assert g.sync_status() == rb.OK      # no key is "out of range"
    g.close()


def test_extreme_keys_and_empty_documents():
    cfg = dict(K=9, B=3, R=2, eta=3, k=31, m=1 << 12)
    o, g = _pair(cfg, 7)
    keys = np.array([0, 1, 2**64 - 1, 2**63, 4**31, 4**31 - 1, 0x5555555555555555], np.uint64)
    offsets = np.array([0, 0, 3, 3, 7, 7, 7, 7, 7, 7], np.uint64)    # empty documents included
    docs = synth.KeyBatch(keys, offsets, np.arange(9, dtype=np.uint32))
    _insert(o, g, docs)
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    q = np.concatenate([keys, np.array([12345, 2**64 - 2], np.uint64)])
    assert np.array_equal(host_u32(g.query_kmers(dev(q, np.int64))), o.query_kmers(q))
    g.close()


def test_raw_key_index_refuses_sequences():
    cfg = dict(K=4, B=2, R=1, eta=1, k=5, m=1024)
    _, g = _pair(cfg, 3)
    s = synth.genome_sets(3, K=4, n_ancestors=1, ancestor_len=50)
    off, ch = dev(s.offsets, np.int64), dev(s.chars, np.uint8)
    with pytest.raises(rb.RamboError) as e:
        g.insert_seqs(dev(s.set_ids, np.int32), off, ch)
    assert e.value.code == rb.EINVAL
    for call in (lambda: g.query_seqs(off, ch), lambda: g.query_seqs_ids(off, ch),
                 lambda: g.extract_kmers(off, ch), lambda: rb.Server(g)):
        with pytest.raises(rb.RamboError):
            call()
    g.close()


def test_wikipedia_sized_index_matches_oracle():
    """The Sec. 5.3 Wikipedia-sample shape: 17 618 documents (about 1.7e7
    distinct document-word pairs), B = 2 000, R = 2, m = 200 000 bits per
    filter.  Sampled rows of both repetitions and 20 000 word queries."""
    cfg = synth.INDEX_WIKI
    docs = synth.config_wiki()
    o, g = _pair(cfg, 2006)
    _insert(o, g, docs)
    rows = np.random.default_rng(5).choice(cfg["m"], size=4000, replace=False)
    for r in range(cfg["R"]):
        assert np.array_equal(gpu_rows(g, r, rows), o.bits_at(r, rows)), r
    q = synth.word_queries(3006, docs, 20_000)
    want = o.query_kmers(q, nthreads=16)
    got = host_u32(g.query_kmers(dev(q, np.int64)))
    assert np.array_equal(got, want)
    g.close()


# Compile-time wide shapes (rows of 256 and 1024 bits, eta = 2) on word
# queries of which many have busy answers, built from the partition with
# the phi loads shared among the wave's terms.
WIDE_BUSY = [
    dict(K=2000, B=200, R=3, eta=2, k=31, m=20_000),
    dict(K=3000, B=250, R=6, eta=2, k=31, m=16_000),
    dict(K=6000, B=600, R=4, eta=2, k=31, m=20_000),
    dict(K=5000, B=1000, R=3, eta=2, k=31, m=12_000),
    dict(K=4000, B=700, R=5, eta=2, k=31, m=12_000),
    dict(K=4000, B=520, R=6, eta=2, k=31, m=12_000),
]


def _partition_share(o, cfg, q):
    """Share of the queries whose answer the kernels build from the
    partition: no repetition empty and the cheaper cell lists still cost
    more than K * R lookups (or over 512 cells)."""
    W = (cfg["K"] + 31) // 32
    hits = 0
    for x in q:
        npos = o.query_cells(int(x)).sum(1)
        if (npos == 0).any():
            continue
        cost = int(np.minimum(npos, cfg["B"] - npos).sum())
        hits += cost > 512 or cost * W > cfg["K"] * cfg["R"]
    return hits / len(q)


@pytest.mark.parametrize("cfg", WIDE_BUSY, ids=lambda c: "K%(K)d-B%(B)d-R%(R)d" % c)
def test_busy_answers_match_oracle(cfg):
    seed = cfg["B"] + 29
    docs = synth.documents(seed, cfg["K"], vocab=5000, median_len=150, min_len=1, max_len=800)
    o, g = _pair(cfg, seed)
    _insert(o, g, docs)
    q = synth.word_queries(seed + 1, docs, 6000, present_frac=0.8)
    assert _partition_share(o, cfg, q[:400]) > 0.1      # the partition path is exercised
    want = o.query_kmers(q, nthreads=8)
    for n in (6000, 4093, 37, 1):                        # many workgroups, ragged, one wave, one term
        got = host_u32(g.query_kmers(dev(q[:n], np.int64)))
        assert np.array_equal(got, want[:n]), n
    g.close()


@pytest.mark.parametrize("cfg", [dict(K=3000, B=2000, R=2, eta=4, k=31, m=4096),
                                 dict(K=6000, B=600, R=4, eta=2, k=31, m=20_000)],
                         ids=["B2000-R2-e4", "B600-R4-e2"])
def test_large_word_batches_match_oracle(cfg):
    # large batches (3e5 terms, tens of thousands of workgroups)
    seed = 7
    docs = synth.documents(seed, cfg["K"], vocab=5000, median_len=150, min_len=1, max_len=800)
    o, g = _pair(cfg, seed)
    _insert(o, g, docs)
    q = synth.word_queries(seed + 1, docs, 300_000, present_frac=0.8)
    want = o.query_kmers(q, nthreads=16)
    assert np.array_equal(host_u32(g.query_kmers(dev(q, np.int64))), want)
    assert np.array_equal(host_u32(g.query_kmers(dev(q[:70_001], np.int64))), want[:70_001])
    g.close()
