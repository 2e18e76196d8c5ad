"""The seeded input generators (host only): deterministic, well-formed, and
the multi-word queries drawn from one document are held by it.  Also the
conjunction that the term-set parity tests compute from the oracle's
per-term answers, pinned against the oracle's own read conjunction
(Sec. 3.2.1) on the k-mers of reads."""
import numpy as np

import oracle
from paper_1910_02611_amd import synth


def test_documents_and_word_sets_are_deterministic_and_well_formed():
    a = synth.documents(5, 120, vocab=3000, median_len=80, min_len=0, max_len=300)
    b = synth.documents(5, 120, vocab=3000, median_len=80, min_len=0, max_len=300)
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.offsets, b.offsets)
    assert a.offsets[0] == 0 and np.all(np.diff(a.offsets.astype(np.int64)) >= 0)
    assert int(a.offsets[-1]) == a.keys.size
    for d in range(a.n):    # distinct words per document
        w = a.keys[int(a.offsets[d]):int(a.offsets[d + 1])]
        assert np.unique(w).size == w.size
    q1 = synth.word_sets(6, a, 500, min_words=0, max_words=6)
    q2 = synth.word_sets(6, a, 500, min_words=0, max_words=6)
    assert np.array_equal(q1.keys, q2.keys) and np.array_equal(q1.offsets, q2.offsets)
    lens = np.diff(q1.offsets.astype(np.int64))
    assert lens.min() >= 0 and lens.max() <= 6 and int(q1.offsets[-1]) == q1.keys.size
    assert np.isin(q1.keys, a.meta["vocab"]).all()


def test_word_sets_from_one_document_are_held_by_it():
    docs = synth.documents(7, 60, vocab=2000, median_len=50, min_len=1, max_len=200)
    sets = [set(docs.keys[int(docs.offsets[d]):int(docs.offsets[d + 1])].tolist()) for d in range(docs.n)]
    q = synth.word_sets(8, docs, 300, min_words=1, max_words=5, from_doc_frac=1.0)
    for i in range(q.n):
        words = set(q.keys[int(q.offsets[i]):int(q.offsets[i + 1])].tolist())
        assert any(words <= s for s in sets), i


def test_conjunction_of_term_answers_is_the_read_answer():
    # the AND of the oracle's per-k-mer answers over a read's valid k-mers
    # equals the oracle's read answer (empty when the read has no k-mer)
    K, B, R, eta, k, m = 40, 8, 3, 2, 15, 1 << 12
    sets = synth.genome_sets(9, K=K, n_ancestors=4, ancestor_len=600)
    o = oracle.OracleIndex(K, B, R, eta, k, m, 9)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 4)
    rd = synth.reads(10, sets, 60, median_len=80, min_len=5, max_len=200, substr_frac=0.7)
    want, nk = o.query_seqs(rd.offsets, rd.chars, nthreads=4)
    codes = oracle.extract(rd.offsets, rd.chars, k)
    for i in range(rd.n):
        c = codes[int(rd.offsets[i]):int(rd.offsets[i + 1])]
        c = c[c != oracle.NO_KMER]
        assert c.size == nk[i]
        got = np.bitwise_and.reduce(o.query_kmers(c), axis=0) if c.size else np.zeros_like(want[i])
        assert np.array_equal(got, want[i]), i
