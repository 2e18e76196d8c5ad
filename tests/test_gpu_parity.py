"""GPU parity: every result of the HIP library equals the oracle's, bit for bit
(all work is integer), on seeded synthetic inputs.  Calls go through the C ABI
(paper_1910_02611_amd.rambo)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_02611_amd import synth
from paper_1910_02611_amd import rambo as rb
from gpu_util import (dev, host_u32, host_u64, make_pair, gpu_insert_seqs, gpu_extract, first_codes_gpu,
                      first_codes_oracle, gpu_index_bits, oracle_index_bits, gpu_rows)

pytestmark = pytest.mark.gpu


def _seqs_with_noise(seed, lengths, k):
    """CSR of random sequences with lower case, N runs and short/empty ones."""
    rng = np.random.default_rng(seed)
    alphabet = np.frombuffer(b"ACGTACGTACGTacgtN", np.uint8)
    parts = [rng.choice(alphabet, size=L) for L in lengths]
    offsets = np.zeros(len(parts) + 1, np.uint64)
    offsets[1:] = np.cumsum([p.size for p in parts])
    chars = np.concatenate(parts).astype(np.uint8) if parts else np.zeros(0, np.uint8)
    return synth.SeqBatch(chars, offsets, np.zeros(len(parts), np.uint32))


@pytest.mark.parametrize("k", [1, 5, 16, 31, 32])
def test_extract_matches_oracle(k):
    lengths = [0, 1, k - 1, k, k + 1, 63, 64, 65, 127, 128, 129, 1000, 0, 3000, 7]
    b = _seqs_with_noise(100 + k, lengths, k)
    _, g = make_pair(dict(K=4, B=2, R=1, eta=1, k=k, m=64), 1)
    got = gpu_extract(g, b)
    want = oracle.extract(b.offsets, b.chars, k)
    assert np.array_equal(got, want)


def test_extract_bytes_outside_sequences():
    # bytes before offsets[0] and after offsets[n] belong to no sequence
    b = _seqs_with_noise(7, [200, 150], 31)
    offsets = b.offsets.copy()
    offsets[0] = 10
    offsets[-1] -= 20
    _, g = make_pair(dict(K=4, B=2, R=1, eta=1, k=31, m=64), 1)
    got = host_u64(g.extract_kmers(dev(offsets, np.int64), dev(b.chars, np.uint8)))
    want = oracle.extract(offsets, b.chars, 31)
    want[:10] = oracle.NO_KMER          # oracle only writes inside the sequences
    want[int(offsets[-1]):] = oracle.NO_KMER
    assert np.array_equal(got, want)


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o, g = make_pair(cfg, seed=2001)
    assert o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8) == 0
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == 0
    return cfg, sets, o, g


def test_partition_table_matches_oracle(tiny):
    _, _, o, g = tiny
    assert np.array_equal(g.partition(), o.phi())


def test_tiny_index_bits_match_oracle(tiny):
    _, _, o, g = tiny
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))


def test_tiny_kmer_queries_match_oracle(tiny):
    cfg, sets, o, g = tiny
    q = synth.kmer_queries(3001, sets, 10_000, cfg["k"])
    codes = first_codes_gpu(g, q)
    ocodes = first_codes_oracle(q, cfg["k"])
    assert np.array_equal(host_u64(codes), ocodes)
    got = host_u32(g.query_kmers(codes))
    want = o.query_kmers(ocodes, nthreads=8)
    assert np.array_equal(got, want)
    # non-canonical orientation and random 62-bit codes
    rng = np.random.default_rng(4)
    rc = rng.integers(0, 1 << 62, size=5000, dtype=np.uint64)
    got = host_u32(g.query_kmers(dev(rc, np.int64)))
    assert np.array_equal(got, o.query_kmers(rc, nthreads=8))


def test_plain_path_matches_batched(tiny):
    cfg, sets, o, g = tiny
    q = synth.kmer_queries(3002, sets, 300, cfg["k"])
    codes = first_codes_gpu(g, q)
    a = host_u32(g.query_kmers(codes))
    b = host_u32(g.query_kmers(codes, plain=True))
    assert np.array_equal(a, b)
    rd = synth.config_batched_reads(sets, 60, seed=3004)
    ma, na = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    mb, nb = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8), plain=True)
    assert np.array_equal(host_u32(ma), host_u32(mb)) and np.array_equal(host_u32(na), host_u32(nb))
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    assert np.array_equal(host_u32(mb), want) and np.array_equal(host_u32(nb), wn.astype(np.uint32))


def test_batched_reads_match_oracle(tiny):
    cfg, sets, o, g = tiny
    rd = synth.config_batched_reads(sets, 3000, seed=3003)
    masks, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    assert np.array_equal(host_u32(nk), wn.astype(np.uint32))
    assert np.array_equal(host_u32(masks), want)
    # true source sets are always reported (zero false negatives)
    got = host_u32(masks)
    src = rd.meta["source_set"]
    for t in np.nonzero(src >= 0)[0][:500]:
        assert (got[t, src[t] // 32] >> (src[t] % 32)) & 1


def test_read_edge_cases(tiny):
    cfg, sets, o, g = tiny
    k = cfg["k"]
    gnm = sets.seq(3)
    reads = [b"", gnm[:k - 1], gnm[:k], gnm[:k + 1], b"N" * 200, gnm[:50] + b"N" + gnm[51:300],
             gnm[:64 + k - 1], gnm[:128 + k], gnm.lower()[:500], gnm, b"ACGT" * 3]
    offsets = np.zeros(len(reads) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(r) for r in reads])
    chars = np.frombuffer(b"".join(reads), np.uint8)
    m, nk = g.query_seqs(dev(offsets, np.int64), dev(chars, np.uint8))
    want, wn = o.query_seqs(offsets, chars)
    assert np.array_equal(host_u32(m), want)
    assert np.array_equal(host_u32(nk), wn.astype(np.uint32))
    assert host_u32(nk)[0] == 0 and not host_u32(m)[0].any()


def test_insert_kmers_path_equals_sequence_path(tiny):
    cfg, sets, o, g = tiny
    codes = oracle.extract(sets.offsets, sets.chars, cfg["k"])
    keep = codes != oracle.NO_KMER
    seg = np.searchsorted(sets.offsets[1:], np.arange(codes.size), side="right")
    offs = np.zeros(sets.n + 1, np.uint64)
    offs[1:] = np.cumsum(np.bincount(seg[keep], minlength=sets.n))
    kc = codes[keep].copy()
    kc[::3] = np.array([oracle.revcomp(int(c), cfg["k"]) for c in kc[::3]], np.uint64)
    _, g2 = make_pair(cfg, seed=2001)
    g2.insert_kmers(dev(sets.set_ids, np.int32), dev(offs, np.int64), dev(kc, np.int64))
    assert g2.sync_status() == 0
    assert torch.equal(g2.index_words(), g.index_words())


def test_streaming_inserts_in_any_order(tiny):
    cfg, sets, o, g = tiny
    _, g2 = make_pair(cfg, seed=2001)
    order = np.random.default_rng(3).permutation(sets.n)
    for part in (order[: sets.n // 3], order[sets.n // 3:]):
        parts = [sets.chars[int(sets.offsets[s]):int(sets.offsets[s + 1])] for s in part]
        offs = np.zeros(len(parts) + 1, np.uint64)
        offs[1:] = np.cumsum([p.size for p in parts])
        b = synth.SeqBatch(np.concatenate(parts), offs, sets.set_ids[part].astype(np.uint32))
        gpu_insert_seqs(g2, b)
    gpu_insert_seqs(g2, sets)   # repeated inserts are idempotent
    assert torch.equal(g2.index_words(), g.index_words())


def test_clear_gives_empty_index(tiny):
    cfg, sets, _, _ = tiny
    _, g2 = make_pair(cfg, seed=2001)
    gpu_insert_seqs(g2, sets)
    g2.clear()
    assert int(g2.index_words().abs().sum()) == 0


def test_device_errors_are_sticky_and_local():
    cfg = dict(K=40, B=5, R=2, eta=2, k=11, m=1 << 12)
    sets = synth.genome_sets(5, K=40, n_ancestors=4, ancestor_len=300)
    o, g = make_pair(cfg, seed=9)
    bad_ids = sets.set_ids.copy()
    bad_ids[7] = 40   # out of range: skipped, flag raised
    o_ids = sets.set_ids.copy()
    keep = np.ones(sets.n, bool)
    keep[7] = False
    for s in np.nonzero(keep)[0]:
        o.insert_seq(int(o_ids[s]), sets.seq(int(s)))
    g.insert_seqs(dev(bad_ids, np.int32), dev(sets.offsets, np.int64), dev(sets.chars, np.uint8))
    assert g.sync_status() == rb.ERANGE
    assert g.sync_status() == 0   # cleared
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    codes = np.array([0, 5, 1 << 22, (1 << 22) - 1, 12345], np.uint64)   # 4^11 = 2^22
    got = host_u32(g.query_kmers(dev(codes, np.int64)))
    assert g.sync_status() == rb.ECODE
    assert not got[2].any()
    for t in (0, 1, 3, 4):
        assert np.array_equal(got[t], o.query_kmer(int(codes[t])))


def test_identity_partition_special_case():
    K = 24
    sets = synth.genome_sets(31, K=K, n_ancestors=3, ancestor_len=500)
    cfg = dict(K=K, B=K, R=1, eta=2, k=21, m=1 << 12)
    o, g = make_pair(cfg, seed=4, flags=oracle.FLAG_IDENTITY_PARTITION)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars)
    gpu_insert_seqs(g, sets)
    assert np.array_equal(g.partition(), np.tile(np.arange(K, dtype=np.uint32), (1, 1)))
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    q = synth.kmer_queries(32, sets, 2000, 21)
    assert np.array_equal(host_u32(g.query_kmers(first_codes_gpu(g, q))),
                          o.query_kmers(first_codes_oracle(q, 21)))


# Shapes covering every row width S (8 .. 4096 bits), the fixed-size and the
# run-time kernels, non-power-of-two m, W > 64 answer words, and k = 32.
SHAPES = [
    dict(K=5, B=5, R=1, eta=1, k=31, m=1000),
    dict(K=70, B=16, R=3, eta=2, k=31, m=1 << 12),
    dict(K=33, B=32, R=2, eta=3, k=21, m=3000),
    dict(K=100, B=50, R=4, eta=2, k=31, m=1 << 13),
    dict(K=300, B=100, R=5, eta=2, k=31, m=5000),
    dict(K=400, B=200, R=5, eta=2, k=31, m=1 << 12),
    dict(K=600, B=500, R=2, eta=1, k=32, m=1 << 11),
    dict(K=2500, B=1000, R=6, eta=2, k=31, m=1 << 11),
    dict(K=3000, B=2000, R=1, eta=4, k=15, m=700),
    dict(K=4100, B=4096, R=2, eta=1, k=31, m=256),
    dict(K=64, B=8, R=7, eta=2, k=31, m=1 << 12),
    dict(K=64, B=8, R=3, eta=1, k=31, m=1 << 12),
    dict(K=4096, B=256, R=3, eta=2, k=31, m=1 << 11),   # answer words a multiple of 4, 2 lanes per query
    dict(K=1024, B=64, R=5, eta=2, k=31, m=1 << 12),    # answer words a multiple of 4, one lane per query
    dict(K=200, B=10, R=16, eta=2, k=31, m=1 << 11),    # the most repetitions, R * eta at its limit of 32
    dict(K=50, B=4, R=2, eta=16, k=27, m=1 << 12),      # the most hashes per filter
]


@pytest.mark.parametrize("cfg", SHAPES, ids=lambda c: "K%(K)d-B%(B)d-R%(R)d-e%(eta)d-k%(k)d-m%(m)d" % c)
def test_shapes_match_oracle(cfg):
    nanc = 5
    K = cfg["K"]
    sets = synth.genome_sets(K + cfg["B"], K=K, n_ancestors=nanc, ancestor_len=400, sub_rate=0.02)
    o, g = make_pair(cfg, seed=cfg["B"] * 7 + cfg["R"])
    assert o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8) == 0
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == 0
    assert np.array_equal(g.partition(), o.phi())
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    q = synth.kmer_queries(K + 1, sets, 700, cfg["k"])
    codes = first_codes_gpu(g, q)
    oc = first_codes_oracle(q, cfg["k"])
    assert np.array_equal(host_u64(codes), oc)
    assert np.array_equal(host_u32(g.query_kmers(codes)), o.query_kmers(oc, nthreads=8))
    rd = synth.reads(K + 2, sets, 120, median_len=120, min_len=1, max_len=400, substr_frac=0.8)
    m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    want, wn = o.query_seqs(rd.offsets, rd.chars, nthreads=8)
    assert np.array_equal(host_u32(nk), wn.astype(np.uint32))
    assert np.array_equal(host_u32(m), want)


def test_zero_sized_calls_are_noops(tiny):
    _, _, _, g = tiny
    e64 = torch.zeros(0, dtype=torch.int64, device="cuda")
    out = g.query_kmers(e64)
    assert out.shape[0] == 0
    g.query_seqs(torch.zeros(1, dtype=torch.int64, device="cuda"), torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert g.sync_status() == 0


# ---------------------------------------------------------------- partitioned insertion

def _partitioned_pair(cfg, seed, scratch=0):
    o, g = make_pair(cfg, seed=seed)
    g.set_insert_policy(rb.INSERT_PARTITIONED, scratch)
    return o, g


def test_partitioned_insert_matches_oracle(tiny):
    cfg, sets, o, _ = tiny
    _, g = _partitioned_pair(cfg, 2001)
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == 0
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))


def test_partitioned_insert_in_many_batches(tiny):
    cfg, sets, o, g_direct = tiny
    _, g = _partitioned_pair(cfg, 2001, scratch=1 << 20)   # ~50k targets per batch
    gpu_insert_seqs(g, sets)
    assert g.sync_status() == 0
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
    assert torch.equal(g.index_words(), g_direct.index_words())


def test_partitioned_insert_reads_back_earlier_bits(tiny):
    # bits set by a direct k-mer insert, and by an earlier partitioned call,
    # survive a later partitioned insert (only the first insert into an
    # all-zero index skips reading the regions back); a clear makes the next
    # insert start from zero again
    cfg, sets, o, g_direct = tiny
    _, g = _partitioned_pair(cfg, 2001)
    half = sets.n // 2
    first = synth.SeqBatch(sets.chars, sets.offsets[:half + 1], sets.set_ids[:half])
    rest_off = sets.offsets[half:]
    rest = synth.SeqBatch(sets.chars, rest_off, sets.set_ids[half:])
    codes = oracle.extract(sets.offsets, sets.chars, cfg["k"])
    seg = np.searchsorted(sets.offsets[1:], np.arange(codes.size), side="right")
    keep = (codes != oracle.NO_KMER) & (seg < half)
    offs = np.zeros(half + 1, np.uint64)
    offs[1:] = np.cumsum(np.bincount(seg[keep], minlength=half))
    g.set_insert_policy(rb.INSERT_DIRECT)
    g.insert_kmers(dev(first.set_ids, np.int32), dev(offs, np.int64), dev(codes[keep].copy(), np.int64))
    g.set_insert_policy(rb.INSERT_PARTITIONED)
    gpu_insert_seqs(g, rest)
    assert torch.equal(g.index_words(), g_direct.index_words())
    g.clear()
    gpu_insert_seqs(g, first)
    gpu_insert_seqs(g, rest)
    assert g.sync_status() == 0
    assert torch.equal(g.index_words(), g_direct.index_words())


def test_partitioned_insert_overflow_falls_back():
    # one k-mer repeated thousands of times crowds one region past its slab
    cfg = dict(K=8, B=4, R=3, eta=2, k=21, m=1 << 16)
    rng = np.random.default_rng(8)
    parts = [np.frombuffer(b"A" * 20000, np.uint8), np.frombuffer(b"ACGT" * 5000, np.uint8)]
    parts += [rng.choice(np.frombuffer(b"ACGT", np.uint8), size=3000) for _ in range(6)]
    offsets = np.zeros(len(parts) + 1, np.uint64)
    offsets[1:] = np.cumsum([p.size for p in parts])
    b = synth.SeqBatch(np.concatenate(parts), offsets, np.arange(len(parts), dtype=np.uint32))
    o, g = _partitioned_pair(cfg, 5, scratch=1 << 20)
    o.insert_seqs(b.set_ids, b.offsets, b.chars)
    gpu_insert_seqs(g, b)
    assert g.sync_status() == 0
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))


@pytest.mark.parametrize("cfg", SHAPES, ids=lambda c: "K%(K)d-B%(B)d-R%(R)d-e%(eta)d-k%(k)d-m%(m)d" % c)
def test_partitioned_shapes_match_oracle(cfg):
    # the partitioned insert (stage A with the targets held in registers for
    # R = 3..6 at eta = 2, the run-time kernel otherwise) against the oracle's
    # separate filters, and against the direct insert
    K = cfg["K"]
    sets = synth.genome_sets(K + cfg["B"] + 1, K=K, n_ancestors=5, ancestor_len=400, sub_rate=0.02)
    o, gd = make_pair(cfg, seed=cfg["B"] * 3 + 1)
    assert o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8) == 0
    gd.set_insert_policy(rb.INSERT_DIRECT)
    _, gp = _partitioned_pair(cfg, cfg["B"] * 3 + 1, scratch=4 << 20)
    gpu_insert_seqs(gd, sets)
    gpu_insert_seqs(gp, sets)
    assert gd.sync_status() == 0 and gp.sync_status() == 0
    want = oracle_index_bits(o)
    assert np.array_equal(gpu_index_bits(gp), want)
    gpu_insert_seqs(gp, sets)   # a second call ORs into the same regions (read back): no change
    assert gp.sync_status() == 0
    assert np.array_equal(gpu_index_bits(gp), want)
    assert np.array_equal(gpu_index_bits(gd), want)


@pytest.mark.parametrize("mis", [0, 1, 3])
@pytest.mark.parametrize("m", [1 << 16, 50_000])
def test_piece_insert_edges(mis, m):
    # the sequence binning kernel's edge cases: sequences shorter than k, of
    # exactly k, around the piece length (8 192 windows) and a lane's span
    # (128 windows), N runs and lower case inside windows, empty sequences,
    # and byte buffers that do not start on a 4-byte boundary; against the
    # oracle, for a power-of-two m (32-bit positions) and another m
    P = 8192
    lengths = [0, 1, 30, 31, 32, 158, 159, 160, P + 29, P + 30, P + 31, 3 * P + 95, 20000, 3, 0, 100_000, 777]
    b = _seqs_with_noise(40 + mis, lengths, 31)
    b.set_ids = (np.arange(b.n) % 40).astype(np.uint32)
    cfg = dict(K=40, B=8, R=4, eta=2, k=31, m=m)
    o, g = _partitioned_pair(cfg, 77 + mis)
    assert o.insert_seqs(b.set_ids, b.offsets, b.chars, 8) == 0
    pad = torch.zeros(b.chars.size + 8, dtype=torch.uint8, device="cuda")
    pad[mis:mis + b.chars.size] = dev(b.chars, np.uint8)
    chars = pad[mis:mis + b.chars.size]
    assert chars.data_ptr() % 4 == mis
    g.insert_seqs(dev(b.set_ids, np.int32), dev(b.offsets, np.int64), chars)
    assert g.sync_status() == 0
    assert np.array_equal(gpu_index_bits(g), oracle_index_bits(o))
