"""GPU parity of the partitioned insert from codes and raw keys (Alg. 1 with
the bit targets sorted into index regions, the same kernels as the sequence
path after stage A): both insert policies give the oracle's index bit for
bit, for k-mer codes (canonical or not) and raw 64-bit keys, in one batch or
many (a small scratch limit), over streaming calls that must read earlier
bits back, and with bad items skipped and reported."""
import numpy as np
import pytest

import oracle
from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import synth
from gpu_util import dev, host_u32, make_pair, gpu_index_bits, oracle_index_bits

pytestmark = pytest.mark.gpu

POLICIES = [rb.INSERT_DIRECT, rb.INSERT_PARTITIONED]


def _kmer_batch(seed, K, k, n_anc=6, anc_len=1500):
    """The k-mer codes of seeded genome sets as a CSR (every third one
    reverse-complemented: the index stores canonical terms)."""
    sets = synth.genome_sets(seed, K=K, n_ancestors=n_anc, ancestor_len=anc_len)
    codes = oracle.extract(sets.offsets, sets.chars, k)
    keep = codes != oracle.NO_KMER
    seg = np.searchsorted(sets.offsets[1:], np.arange(codes.size), side="right")
    offs = np.zeros(sets.n + 1, np.uint64)
    offs[1:] = np.cumsum(np.bincount(seg[keep], minlength=sets.n))
    kc = codes[keep].copy()
    kc[::3] = np.array([oracle.revcomp(int(c), k) for c in kc[::3]], np.uint64)
    return synth.KeyBatch(kc, offs, sets.set_ids.astype(np.uint32))


def _split(b, at):
    """The first `at` sets and the rest, as two batches."""
    o = b.offsets
    first = synth.KeyBatch(b.keys[: int(o[at])], o[: at + 1].copy(), b.set_ids[:at])
    rest = synth.KeyBatch(b.keys[int(o[at]):], o[at:] - o[at], b.set_ids[at:])
    return first, rest


def _gpu_insert(g, b):
    g.insert_kmers(dev(b.set_ids, np.int32), dev(b.offsets, np.int64), dev(b.keys, np.int64))


CASES = [
    # (index shape, raw keys)
    (dict(K=300, B=40, R=4, eta=2, k=31, m=1 << 15), False),
    (dict(K=200, B=50, R=3, eta=2, k=21, m=20_000), False),
    (dict(K=2000, B=300, R=2, eta=4, k=31, m=50_000), True),    # the documents shape
    (dict(K=500, B=100, R=6, eta=2, k=31, m=9000), True),
    (dict(K=400, B=64, R=4, eta=3, k=31, m=1 << 14), True),     # run-time shape: the generic stage A
    (dict(K=150, B=30, R=1, eta=5, k=25, m=1 << 13), False),
]


@pytest.mark.parametrize("policy", POLICIES, ids=["direct", "partitioned"])
@pytest.mark.parametrize("cfg,raw", CASES, ids=lambda c: str(c) if isinstance(c, bool) else
                         "R%(R)d-e%(eta)d-B%(B)d-m%(m)d" % c)
def test_code_insert_matches_oracle(cfg, raw, policy):
    seed = cfg["B"] + cfg["R"]
    flags = oracle.FLAG_RAW_KEYS if raw else 0
    o, g = make_pair(cfg, seed=seed, flags=flags)
    if raw:
        b = synth.documents(seed, cfg["K"], vocab=30_000, median_len=60, min_len=0, max_len=400)
    else:
        b = _kmer_batch(seed, cfg["K"], cfg["k"])
    assert o.insert_kmers(b.set_ids, b.offsets, b.keys, 8) == 0
    # a scratch of 1 MiB holds about 2e5 targets: several batches
    g.set_insert_policy(policy, 1 << 20)
    first, rest = _split(b, len(b.set_ids) // 3)
    _gpu_insert(g, first)           # into the all-zero index
    _gpu_insert(g, rest)            # reads the first call's bits back
    assert g.sync_status() == rb.OK
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    _gpu_insert(g, b)               # idempotent
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    q = b.keys[:: max(1, b.keys.size // 3000)]
    assert np.array_equal(host_u32(g.query_kmers(dev(q, np.int64))), o.query_kmers(q, nthreads=8))
    g.close()


@pytest.mark.parametrize("policy", POLICIES, ids=["direct", "partitioned"])
def test_bad_codes_and_set_ids_are_skipped(policy):
    cfg = dict(K=100, B=20, R=4, eta=2, k=15, m=1 << 14)
    b = _kmer_batch(17, cfg["K"], cfg["k"], n_anc=4, anc_len=800)
    o, g = make_pair(cfg, seed=17)
    keys = b.keys.copy()
    bad = np.zeros(keys.size, bool)
    bad[5::97] = True
    keys[bad] = (1 << 30) + np.arange(bad.sum(), dtype=np.uint64)    # >= 4^15
    good_off = np.zeros_like(b.offsets)
    seg = np.searchsorted(b.offsets[1:], np.arange(keys.size), side="right")
    good_off[1:] = np.cumsum(np.bincount(seg[~bad], minlength=len(b.set_ids)))
    assert o.insert_kmers(b.set_ids, good_off, b.keys[~bad], 4) == 0
    g.set_insert_policy(policy)
    g.insert_kmers(dev(b.set_ids, np.int32), dev(b.offsets, np.int64), dev(keys, np.int64))
    assert g.sync_status() == rb.ECODE
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    ids = b.set_ids.copy()
    ids[3] = cfg["K"]               # out of range: that set's codes are skipped
    g.insert_kmers(dev(ids, np.int32), dev(good_off, np.int64), dev(b.keys[~bad], np.int64))
    assert g.sync_status() == rb.ERANGE
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    g.close()


def test_partitioned_code_insert_after_fold_and_clear():
    # the scratch is re-planned for the folded index (B -> B/2); a clear makes
    # the next insert start from an all-zero index again
    cfg = dict(K=600, B=200, R=2, eta=4, k=31, m=30_000)
    docs = synth.documents(23, cfg["K"], vocab=20_000, median_len=50, min_len=1, max_len=300)
    o, g = make_pair(cfg, seed=23, flags=oracle.FLAG_RAW_KEYS)
    g.set_insert_policy(rb.INSERT_PARTITIONED)
    first, rest = _split(docs, cfg["K"] // 2)
    o.insert_kmers(first.set_ids, first.offsets, first.keys, 4)
    _gpu_insert(g, first)
    o.fold()
    g.fold()
    o.insert_kmers(rest.set_ids, rest.offsets, rest.keys, 4)
    _gpu_insert(g, rest)
    assert g.sync_status() == rb.OK
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    g.clear()
    o2, _ = make_pair(cfg, seed=23, flags=oracle.FLAG_RAW_KEYS)
    o2.fold()
    o2.insert_kmers(rest.set_ids, rest.offsets, rest.keys, 4)
    _gpu_insert(g, rest)
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o2))
    g.close()
