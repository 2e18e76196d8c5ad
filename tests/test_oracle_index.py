"""Pins of the oracle index (Alg. 1, Alg. 2, Sec. 3.2.1) against what the paper
and the mathematics fix:

* zero false negatives against brute-force exact MSMT (Sec. 4.1);
* a near-perfect filter (huge m, tiny sets) must return exactly the sets whose
  cell holds a true set in every repetition, the closed form of Alg. 2 when no
  Bloom filter errs;
* B = K with one set per cell and R = 1 is an array of Bloom filters (Sec. 4.3);
  B = 1 is one Bloom filter of the union;
* per-cell fill against the occupancy law behind Sec. 2's FPR formula;
* the measured false-positive rate against Lemma 4.1 (conditioned on the
  realised partition and fills) within 3 sigma, for random and present
  queries and for a planted-multiplicity grid (the Sec. 5.2 protocol);
* sequence answers (Sec. 3.2.1) against brute force.
"""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from oracle import fpr
from paper_1910_02611_amd import synth


def build_oracle(sets, cfg, seed, flags=0, nthreads=4):
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed, flags)
    assert o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, nthreads) == 0
    return o


def exact_index(sets, k):
    ex = bf.ExactMSMT(k)
    for s in range(sets.n):
        ex.add_seq(int(sets.set_ids[s]), sets.seq(s))
    return ex


def query_codes(q: synth.SeqBatch, k):
    codes = oracle.extract(q.offsets, q.chars, k)
    return codes[q.offsets[:-1].astype(np.int64)]


@pytest.fixture(scope="module")
def tiny():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o = build_oracle(sets, cfg, seed=2001)
    ex = exact_index(sets, cfg["k"])
    return cfg, sets, o, ex


def test_tiny_zero_false_negatives(tiny):
    cfg, sets, o, ex = tiny
    q = synth.kmer_queries(3001, sets, 10_000, cfg["k"])
    codes = query_codes(q, cfg["k"])
    masks = o.query_kmers(codes, nthreads=4)
    n_fp_random = 0
    for t in range(q.n):
        truth = ex.query_kmer(q.seq(t))
        got = set(oracle.mask_to_ids(masks[t], cfg["K"]))
        assert truth <= got, t
        if q.meta["present"][t]:
            assert truth
        else:
            n_fp_random += len(got - truth)
    # random terms: about p^R per set (Lemma 4.1 with V = 0), p ~ 0.05 here
    assert n_fp_random < 0.002 * (q.n // 2) * cfg["K"]


def test_streaming_and_order_independence(tiny):
    cfg, sets, o, _ = tiny
    o2 = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2001)
    order = np.random.default_rng(1).permutation(sets.n)
    for s in order:  # one set at a time, shuffled, single-sequence path
        o2.insert_seq(int(sets.set_ids[s]), sets.seq(int(s)))
    # and once more: repeated inserts are idempotent
    o2.insert_seq(int(sets.set_ids[order[0]]), sets.seq(int(order[0])))
    for r in range(cfg["R"]):
        for b in range(cfg["B"]):
            assert (o.bfu_words(r, b) == o2.bfu_words(r, b)).all()


def test_kmer_insert_path_equals_sequence_path(tiny):
    cfg, sets, o, _ = tiny
    codes = oracle.extract(sets.offsets, sets.chars, cfg["k"])
    keep = codes != oracle.NO_KMER
    seg = np.searchsorted(sets.offsets[1:], np.arange(codes.size), side="right")
    offs = np.zeros(sets.n + 1, np.uint64)
    offs[1:] = np.cumsum(np.bincount(seg[keep], minlength=sets.n))
    o2 = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2001)
    # non-canonical orientation on purpose: insertion canonicalises
    kc = codes[keep]
    rc = np.array([oracle.revcomp(int(c), cfg["k"]) for c in kc[:5000]], np.uint64)
    kc = kc.copy()
    kc[:5000] = rc
    assert o2.insert_kmers(sets.set_ids, offs, kc, 4) == 0
    assert (o.fill_counts() == o2.fill_counts()).all()
    for r in range(cfg["R"]):
        for b in range(cfg["B"]):
            assert (o.bfu_words(r, b) == o2.bfu_words(r, b)).all()


def _closed_form_answer(phi, truth):
    """Alg. 2 with error-free Bloom filters: i is returned iff in every
    repetition its cell also holds one of the true sets."""
    R, K = phi.shape
    if not truth:
        return set()
    cells = [{int(phi[r, j]) for j in truth} for r in range(R)]
    return {i for i in range(K) if all(int(phi[r, i]) in cells[r] for r in range(R))}


def test_near_perfect_filter_equals_closed_form():
    cfg = dict(K=24, B=4, R=3, eta=2, k=15, m=1 << 22)
    sets = synth.genome_sets(77, K=24, n_ancestors=3, ancestor_len=300, sub_rate=0.02)
    o = build_oracle(sets, cfg, seed=5)
    ex = exact_index(sets, cfg["k"])
    phi = o.phi()
    q = synth.kmer_queries(78, sets, 3000, cfg["k"], present_frac=0.7)
    codes = query_codes(q, cfg["k"])
    masks = o.query_kmers(codes)
    for t in range(q.n):
        w = q.seq(t)
        truth = ex.query_kmer(w)
        want = _closed_form_answer(phi, truth)
        assert set(oracle.mask_to_ids(masks[t], cfg["K"])) == want
        # the reverse complement is the same term
        rcm = o.query_kmer(bf.code_of_str(bf.revcomp_str(w)))
        assert (rcm == masks[t]).all()
        # Alg. 2's cell tests: exactly the cells holding a true set
        G = o.query_cells(int(codes[t]))
        for r in range(cfg["R"]):
            assert set(np.nonzero(G[r])[0].tolist()) == {int(phi[r, j]) for j in truth}


def test_array_of_bloom_filters_special_case():
    """B = K, identity partition, R = 1: cell i is the Bloom filter of S_i."""
    K = 16
    sets = synth.genome_sets(91, K=K, n_ancestors=4, ancestor_len=400, sub_rate=0.01)
    cfg = dict(K=K, B=K, R=1, eta=2, k=21, m=1 << 21)
    o = build_oracle(sets, cfg, seed=9, flags=oracle.FLAG_IDENTITY_PARTITION)
    ex = exact_index(sets, cfg["k"])
    q = synth.kmer_queries(92, sets, 2000, cfg["k"])
    masks = o.query_kmers(query_codes(q, cfg["k"]))
    for t in range(q.n):
        assert set(oracle.mask_to_ids(masks[t], K)) == ex.query_kmer(q.seq(t))
    # with a small m the same structure has per-set FPR p of Sec. 2
    cfg2 = dict(cfg, m=1 << 12)
    o2 = build_oracle(sets, cfg2, seed=9, flags=oracle.FLAG_IDENTITY_PARTITION)
    rq = synth.kmer_queries(93, sets, 20000, cfg["k"], present_frac=0.0)
    rm = o2.query_kmers(query_codes(rq, cfg["k"]))
    n_set = ex.distinct_per_set(K)
    bits = np.unpackbits(rm.view(np.uint8), axis=1, bitorder="little")[:, :K]
    for i in range(K):
        p = fpr.bf_fpr(n_set[i], cfg2["m"], 2)
        obs = bits[:, i].mean()
        se = np.sqrt(p * (1 - p) / rq.n)
        assert abs(obs - p) < 4 * se + 2e-3, (i, obs, p)


def test_single_cell_is_one_bloom_filter_of_the_union():
    sets = synth.genome_sets(55, K=10, n_ancestors=2, ancestor_len=200)
    cfg = dict(K=10, B=1, R=2, eta=2, k=11, m=1 << 16)
    o = build_oracle(sets, cfg, seed=3)
    ex = exact_index(sets, cfg["k"])
    q = synth.kmer_queries(56, sets, 500, cfg["k"])
    masks = o.query_kmers(query_codes(q, cfg["k"]))
    for t in range(q.n):
        ids = oracle.mask_to_ids(masks[t], 10)
        assert ids in ([], list(range(10)))
        if ex.query_kmer(q.seq(t)):
            assert ids == list(range(10))


def test_fill_matches_occupancy_law(tiny):
    cfg, sets, o, ex = tiny
    phi = o.phi()
    fill = o.fill_counts()
    zs = []
    for r in range(cfg["R"]):
        n_b = ex.distinct_per_cell(phi[r], cfg["B"])
        for b in range(cfg["B"]):
            e0, v0 = fpr.occupancy_zero_bits_moments(cfg["eta"] * n_b[b], cfg["m"])
            zeros = cfg["m"] - int(fill[r, b])
            zs.append((zeros - e0) / np.sqrt(v0))
    zs = np.array(zs)
    assert np.abs(zs).max() < 4.0, zs
    assert abs(zs.mean()) < 4.0 / np.sqrt(zs.size) + 0.5


def _fp_counts(masks, truths, K):
    bits = np.unpackbits(masks.view(np.uint8), axis=1, bitorder="little")[:, :K]
    obs = bits.sum(axis=1).astype(np.float64)
    tcount = np.array([len(t) for t in truths], np.float64)
    return obs - tcount


def test_fpr_lemma41_random_queries(tiny):
    cfg, sets, o, ex = tiny
    K = cfg["K"]
    phi = o.phi()
    pcell = fpr.cell_fpr(o.fill_counts(), cfg["m"], cfg["eta"])
    rng = np.random.default_rng(17)
    n = 400_000
    codes = rng.integers(0, 1 << 62, size=n, dtype=np.uint64)
    masks = o.query_kmers(codes, nthreads=8)
    truths = [set()] * n   # random 31-mers: collision odds ~ 1e-13 per query
    pr = fpr.report_probability(phi, pcell, [])
    exp = np.full(n, pr.sum())
    obs = _fp_counts(masks, truths, K)
    o_fpr, p_fpr, z = fpr.fpr_gate(obs, exp, np.full(n, K))
    assert abs(z) < 3.0, (o_fpr, p_fpr, z)
    # Lemma 4.1 with V = 0 reduces to p^R; the conditional form averages to it
    p_mean = pcell.mean()
    assert fpr.lemma41(p_mean, cfg["B"], 0, cfg["R"]) == pytest.approx(p_mean ** cfg["R"])


def test_fpr_lemma41_present_queries(tiny):
    cfg, sets, o, ex = tiny
    K = cfg["K"]
    phi = o.phi()
    pcell = fpr.cell_fpr(o.fill_counts(), cfg["m"], cfg["eta"])
    q = synth.kmer_queries(3101, sets, 40_000, cfg["k"], present_frac=1.0)
    masks = o.query_kmers(query_codes(q, cfg["k"]), nthreads=8)
    truths = [ex.query_kmer(q.seq(t)) for t in range(q.n)]
    exp = np.array([fpr.report_probability(phi, pcell, t).sum() - len(t) for t in truths])
    obs = _fp_counts(masks, truths, K)
    neg = np.array([K - len(t) for t in truths])
    o_fpr, p_fpr, z = fpr.fpr_gate(obs, exp, neg)
    assert abs(z) < 3.0, (o_fpr, p_fpr, z)
    assert o_fpr > 0.01   # sibling genomes share cells: the separability term


def test_fpr_planted_multiplicity_grid(tiny):
    """Sec. 5.2 protocol: fresh random terms planted in V random sets."""
    cfg, sets, _, _ = tiny
    K, B, R = cfg["K"], cfg["B"], cfg["R"]
    o = build_oracle(sets, cfg, seed=2001)
    rng = np.random.default_rng(23)
    grid = [1, 2, 4, 8, 16, 32]
    per_v = 1500
    planted = []
    for V in grid:
        for _ in range(per_v):
            code = int(rng.integers(0, 1 << 62, dtype=np.uint64))
            holders = set(int(i) for i in rng.choice(K, size=V, replace=False))
            for i in holders:
                assert o.insert_kmer(i, code) == 0
            planted.append((V, code, holders))
    phi = o.phi()
    pcell = fpr.cell_fpr(o.fill_counts(), cfg["m"], cfg["eta"])
    codes = np.array([c for _, c, _ in planted], np.uint64)
    masks = o.query_kmers(codes, nthreads=8)
    truths = [h for _, _, h in planted]
    for t in range(len(planted)):   # zero false negatives
        assert truths[t] <= set(oracle.mask_to_ids(masks[t], K))
    obs = _fp_counts(masks, truths, K)
    exp = np.array([fpr.report_probability(phi, pcell, h).sum() - len(h) for h in truths])
    neg = np.array([K - len(h) for h in truths])
    rates = []
    for gi, V in enumerate(grid):
        sl = slice(gi * per_v, (gi + 1) * per_v)
        o_fpr, p_fpr, z = fpr.fpr_gate(obs[sl], exp[sl], neg[sl])
        assert abs(z) < 3.0, (V, o_fpr, p_fpr, z)
        rates.append(o_fpr)
        # unconditional Lemma 4.1 (averaged over partitions) is the same order
        lem = fpr.lemma41(pcell.mean(), B, V, R)
        assert 0.3 * lem < p_fpr < 3.0 * lem + 1e-3, (V, p_fpr, lem)
    assert all(rates[i] < rates[i + 1] for i in range(len(rates) - 1))


def test_sequence_queries_against_bruteforce(tiny):
    cfg, sets, o, ex = tiny
    rd = synth.reads(3003, sets, 400, median_len=200, min_len=20, max_len=2000, substr_frac=0.7)
    masks, nk = o.query_seqs(rd.offsets, rd.chars, nthreads=4)
    for t in range(rd.n):
        s = rd.seq(t)
        truth = ex.query_seq(s)
        got = set(oracle.mask_to_ids(masks[t], cfg["K"]))
        assert int(nk[t]) == len(bf.kmers_of(s, cfg["k"]))
        if truth is None:
            assert not got and nk[t] == 0
        else:
            assert truth <= got
        if rd.meta["source_set"][t] >= 0 and len(s) >= cfg["k"]:
            assert int(rd.meta["source_set"][t]) in got


def test_sequence_query_near_perfect_filter():
    cfg = dict(K=24, B=4, R=3, eta=2, k=15, m=1 << 22)
    sets = synth.genome_sets(77, K=24, n_ancestors=3, ancestor_len=300, sub_rate=0.02)
    o = build_oracle(sets, cfg, seed=5)
    ex = exact_index(sets, cfg["k"])
    phi = o.phi()
    rd = synth.reads(79, sets, 300, median_len=40, min_len=5, max_len=300, substr_frac=0.8)
    masks, nk = o.query_seqs(rd.offsets, rd.chars)
    for t in range(rd.n):
        s = rd.seq(t)
        ks = bf.kmers_of(s, cfg["k"])
        want = set(range(cfg["K"])) if ks else set()
        for w in ks:
            want &= _closed_form_answer(phi, ex.query_kmer(w))
        assert set(oracle.mask_to_ids(masks[t], cfg["K"])) == want
        assert int(nk[t]) == len(ks)


def test_sequence_query_edge_cases(tiny):
    cfg, sets, o, _ = tiny
    k = cfg["k"]
    g = sets.seq(5)
    # shorter than k, exactly k, k with an N, only N
    m0, n0 = o.query_seq(g[:k - 1])
    assert n0 == 0 and not m0.any()
    m1, n1 = o.query_seq(g[:k])
    assert n1 == 1 and (m1 == o.query_kmer(oracle.encode_kmer(g[:k]))).all()
    m2, n2 = o.query_seq(g[:3] + b"N" + g[4:k + 8])   # windows 4..8 are valid
    assert n2 == 5
    m3, n3 = o.query_seq(b"N" * 100)
    assert n3 == 0 and not m3.any()
    # lower case is the same sequence
    m4, _ = o.query_seq(g[100:400].lower())
    m5, _ = o.query_seq(g[100:400])
    assert (m4 == m5).all() and 5 in oracle.mask_to_ids(m5, cfg["K"])


def test_out_of_range_inputs(tiny):
    cfg, _, o, _ = tiny
    assert o.insert_kmer(cfg["K"], 0) != 0
    assert o.insert_kmer(0, 1 << 62) != 0
    assert not o.query_kmer(1 << 62).any()
    bad = np.array([cfg["K"]], np.uint32)
    assert o.insert_seqs(bad, np.array([0, 40], np.uint64), np.frombuffer(b"A" * 40, np.uint8)) != 0


# ----------------------------------------------- rows of large indexes

def _rows_from_filters(o, D=1):
    """[R, m/D, B] bits of the full oracle's filters at positions p % D == 0."""
    out = np.zeros((o.R, o.m // D, o.B), np.uint8)
    for r in range(o.R):
        for b in range(o.B):
            out[r, :, b] = o.bfu_bits(r, b)[::D]
    return out


def _unpack_rows(words, B):
    bits = np.unpackbits(words.view(np.uint8), bitorder="little").reshape(words.shape[:-1] + (-1,))
    return bits[..., :B]


@pytest.mark.parametrize("cfg", [dict(K=64, B=8, R=3, eta=2, k=31, m=1 << 12),
                                 dict(K=300, B=130, R=2, eta=3, k=21, m=1 << 10)])
def test_row_scan_equals_filters(cfg):
    # the row view computed from Alg. 1's definition in one pass equals the
    # transposed filters of the full oracle, for sampled rows and listed keys
    sets = synth.genome_sets(77, K=cfg["K"], n_ancestors=4, ancestor_len=300, sub_rate=0.02)
    full = oracle.OracleIndex(**cfg, seed=91)
    full.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 4)
    lean = oracle.OracleIndex(**cfg, seed=91, flags=oracle.FLAG_NO_FILTERS)
    assert lean.insert_seqs(sets.set_ids, sets.offsets, sets.chars) != 0   # no filters to insert into
    want = _rows_from_filters(full)
    for D in (1, 8):
        sampled, _ = lean.scan_rows(sets.set_ids, sets.offsets, sets.chars, D=D, nthreads=4)
        assert np.array_equal(_unpack_rows(sampled, cfg["B"]), want[:, ::D, :])
    rng = np.random.default_rng(5)
    keys = np.unique(rng.integers(0, cfg["R"] * cfg["m"], size=300).astype(np.uint64))
    _, rows = lean.scan_rows(sets.set_ids, sets.offsets, sets.chars, keys=keys, nthreads=4)
    got = _unpack_rows(rows, cfg["B"])
    for t, key in enumerate(keys):
        r, p = divmod(int(key), cfg["m"])
        assert np.array_equal(got[t], want[r, p])


def test_read_answers_from_rows_equal_full_oracle():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    full = oracle.OracleIndex(**cfg, seed=2001)
    full.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    lean = oracle.OracleIndex(**cfg, seed=2001, flags=oracle.FLAG_NO_FILTERS)
    rd = synth.reads(3021, sets, 150, median_len=150, min_len=20, max_len=400, substr_frac=0.8, read_sub_rate=0.01)
    keys = np.unique(lean.window_keys(rd.offsets, rd.chars))
    _, rows = lean.scan_rows(sets.set_ids, sets.offsets, sets.chars, keys=keys, nthreads=8)
    got, gk = lean.query_seqs_rows(rd.offsets, rd.chars, keys, rows, nthreads=8)
    want, wk = full.query_seqs(rd.offsets, rd.chars, nthreads=8)
    assert np.array_equal(gk, wk)
    assert np.array_equal(got, want)
    with pytest.raises(ValueError):   # a row it was not given
        lean.query_seqs_rows(rd.offsets, rd.chars, keys[1:], rows[1:])


def test_cell_bits_and_members_equal_full_oracle():
    # one cell's BFU from the sets it holds equals that filter of the full
    # oracle, and a set's membership in read answers decided from its R cells
    # equals its bit in the full oracle's answers (reads with substitutions,
    # random reads, reads shorter than k and reads with no valid window)
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    full = oracle.OracleIndex(**cfg, seed=2001)
    full.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    lean = oracle.OracleIndex(**cfg, seed=2001, flags=oracle.FLAG_NO_FILTERS)
    for r in range(cfg["R"]):
        for b in range(cfg["B"]):
            got = lean.cell_bits(r, b, sets.set_ids, sets.offsets, sets.chars, nthreads=4)
            assert np.array_equal(got, full.bfu_words(r, b)), (r, b)
    rd = synth.reads(3022, sets, 120, median_len=100, min_len=20, max_len=300, substr_frac=0.7, read_sub_rate=0.01)
    extra = [b"ACGTN" * 12, b"ACGT" * 5]   # a window broken every 5 bases; shorter than k
    chars = np.concatenate([rd.chars] + [np.frombuffer(e, np.uint8) for e in extra])
    offsets = np.concatenate([rd.offsets, rd.offsets[-1] + np.cumsum([len(e) for e in extra])]).astype(np.uint64)
    want, _ = full.query_seqs(offsets, chars, nthreads=4)
    phi = lean.phi()
    n_pos = 0
    src = rd.meta["source_set"]
    for s in sorted(set(sets.set_ids[src[src >= 0][:4]].tolist()) | {0, cfg["K"] - 1}):
        cells = [lean.cell_bits(r, int(phi[r, s]), sets.set_ids, sets.offsets, sets.chars) for r in range(cfg["R"])]
        got = lean.members_from_cells(offsets, chars, cells)
        bit = ((want[:, s // 32] >> np.uint32(s % 32)) & 1).astype(bool)
        assert np.array_equal(got, bit), s
        assert not got[-2:].any()
        n_pos += int(got.sum())
    assert n_pos > 0
    with pytest.raises(ValueError):
        lean.cell_bits(cfg["R"], 0, sets.set_ids, sets.offsets, sets.chars)


# ------------------------------------------------------------ folding over

@pytest.mark.parametrize("B", [8, 50])
def test_fold_equals_index_built_with_halved_partition(B):
    # folding over (OR of cell b + B/2 into cell b) gives the index that the
    # partition phi mod (B/2) builds directly, bit for bit, and its answers
    cfg = dict(K=120, B=B, R=3, eta=2, k=31, m=1 << 12)
    sets = synth.genome_sets(501, K=120, n_ancestors=6, ancestor_len=400, sub_rate=0.02)
    folded = oracle.OracleIndex(**cfg, seed=77)
    folded.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 4)
    phi = folded.phi().copy()
    folded.fold()
    assert folded.B == B // 2
    assert np.array_equal(folded.phi(), phi % (B // 2))
    direct = oracle.OracleIndex(**dict(cfg, B=B // 2), seed=77)
    direct.set_partition(phi % (B // 2))
    direct.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 4)
    for r in range(cfg["R"]):
        for b in range(B // 2):
            assert np.array_equal(folded.bfu_words(r, b), direct.bfu_words(r, b))
    rd = synth.reads(502, sets, 100, median_len=80, min_len=31, max_len=300, substr_frac=0.7)
    assert np.array_equal(folded.query_seqs(rd.offsets, rd.chars)[0], direct.query_seqs(rd.offsets, rd.chars)[0])
    # folding never loses a holder: truth is still inside every answer
    exact = bf.ExactMSMT(cfg["k"])
    for i in range(sets.n):
        exact.add_seq(int(sets.set_ids[i]), sets.seq(i))
    answers = folded.query_seqs(rd.offsets, rd.chars)[0]
    for q in range(rd.n):
        truth = exact.query_seq(rd.seq(q))
        if truth is not None:
            assert truth <= set(oracle.mask_to_ids(answers[q], cfg["K"]))


# --------------------------------------------------- raw 64-bit keys (Sec. 5.3)

def test_raw_key_sets_exactly_its_positions():
    # one key outside any k-mer range, in one set: every repetition's cell of
    # that set holds exactly the eta multiply-shift positions of the key
    # itself (no canonical form, no range check); every other cell is empty
    cfg = dict(K=6, B=3, R=3, eta=3, k=5, m=4096)
    o = oracle.OracleIndex(**cfg, seed=91, flags=oracle.FLAG_RAW_KEYS)
    x = (1 << 63) + 12345
    assert o.insert_kmers(np.array([4], np.uint32), np.array([0, 1], np.uint64), np.array([x], np.uint64)) == 0
    _, _, s, phi = o.params()
    for r in range(cfg["R"]):
        for b in range(cfg["B"]):
            want = np.zeros(cfg["m"], np.uint8)
            if b == phi[r, 4]:
                want[[oracle.position(x, int(s[r, j]), cfg["m"]) for j in range(cfg["eta"])]] = 1
            assert np.array_equal(o.bfu_bits(r, b), want), (r, b)


def test_raw_keys_are_not_canonicalised():
    # a k-mer code and its reverse complement are one term of a k-mer index
    # but two keys of a raw-key index
    k = 11
    code = oracle.encode_kmer(b"ACGTTGCAAAC")
    rc = oracle.revcomp(code, k)
    assert rc != code
    cfg = dict(K=4, B=2, R=2, eta=2, k=k, m=1 << 16)
    one = lambda c: (np.array([1], np.uint32), np.array([0, 1], np.uint64), np.array([c], np.uint64))
    km = oracle.OracleIndex(**cfg, seed=5)
    raw = oracle.OracleIndex(**cfg, seed=5, flags=oracle.FLAG_RAW_KEYS)
    km.insert_kmers(*one(rc))
    raw.insert_kmers(*one(oracle.canonical(code, k)))
    same = all(np.array_equal(km.bfu_words(r, b), raw.bfu_words(r, b)) for r in range(2) for b in range(2))
    assert same                       # canonical code as a raw key = the k-mer term
    raw2 = oracle.OracleIndex(**cfg, seed=5, flags=oracle.FLAG_RAW_KEYS)
    raw2.insert_kmers(*one(max(code, rc)))
    assert not all(np.array_equal(raw2.bfu_words(r, b), raw.bfu_words(r, b)) for r in range(2) for b in range(2))


def test_raw_key_index_equals_kmer_index_on_canonical_codes():
    # inserting every window's canonical code as a raw key builds the same
    # filters as inserting the sequences (Alg. 1 over the same terms)
    cfg = dict(K=30, B=6, R=3, eta=2, k=21, m=1 << 14)
    sets = synth.genome_sets(93, K=30, n_ancestors=3, ancestor_len=300)
    km = build_oracle(sets, cfg, 17)
    codes = oracle.extract(sets.offsets, sets.chars, cfg["k"])
    keep = codes != oracle.NO_KMER
    seg = np.repeat(np.arange(sets.n), sets.lengths().astype(np.int64))
    off = np.zeros(sets.n + 1, np.uint64)
    np.cumsum(np.bincount(seg[keep], minlength=sets.n), out=off[1:])
    raw = oracle.OracleIndex(**cfg, seed=17, flags=oracle.FLAG_RAW_KEYS)
    assert raw.insert_kmers(sets.set_ids, off, codes[keep], 4) == 0
    for r in range(cfg["R"]):
        for b in range(cfg["B"]):
            assert np.array_equal(raw.bfu_words(r, b), km.bfu_words(r, b))


def test_raw_key_documents_no_false_negatives_and_exact_when_filters_are_perfect():
    # documents as sets of word keys: every document holding a word is in its
    # answer (Sec. 4.1); with filters far larger than the sets, the answer is
    # exactly the documents whose cell holds a true holder in every
    # repetition (Alg. 2 with no Bloom-filter error)
    docs = synth.documents(95, 60, vocab=3000, median_len=60, min_len=5, max_len=400)
    cfg = dict(K=60, B=8, R=3, eta=3, k=31, m=1 << 22)
    o = oracle.OracleIndex(**cfg, seed=19, flags=oracle.FLAG_RAW_KEYS)
    assert o.insert_kmers(docs.set_ids, docs.offsets, docs.keys, 4) == 0
    holders = {}
    for d in range(docs.n):
        for x in docs.keys[int(docs.offsets[d]):int(docs.offsets[d + 1])].tolist():
            holders.setdefault(x, set()).add(d)
    q = synth.word_queries(96, docs, 2000)
    got = o.query_kmers(q, nthreads=4)
    phi = o.phi()
    for t, x in enumerate(q.tolist()):
        ids = set(oracle.mask_to_ids(got[t], cfg["K"]))
        true = holders.get(x, set())
        assert true <= ids
        cells = [{int(phi[r, i]) for i in true} for r in range(cfg["R"])]
        want = {i for i in range(cfg["K"]) if all(int(phi[r, i]) in cells[r] for r in range(cfg["R"]))}
        assert ids == want


def test_raw_key_index_refuses_sequences():
    cfg = dict(K=4, B=2, R=1, eta=1, k=5, m=64)
    o = oracle.OracleIndex(**cfg, seed=1, flags=oracle.FLAG_RAW_KEYS)
    s = synth.genome_sets(3, K=4, n_ancestors=1, ancestor_len=50)
    assert o.insert_seqs(s.set_ids, s.offsets, s.chars) != 0
    with pytest.raises(ValueError):
        o.query_seqs(s.offsets, s.chars)
