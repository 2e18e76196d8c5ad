"""The parameter helper (host only) against the formulas it restates and
against the oracle: the suggested filter size reaches the target
false-positive rate on a built index."""
import math

import numpy as np
import pytest

import oracle
from paper_1910_02611_amd import params, synth


def test_bloom_optimum_reaches_p():
    # at eta = -log2 p and m = -n ln p / (ln 2)^2 the rate is p (up to the
    # rounding of eta): the (ln 2)^2 divisor is what makes the optimum hold
    for p in (0.1, 0.01, 0.001, 1e-5):
        n = 10 ** 6
        eta, m = params.bloom_hashes(p), params.bloom_bits(n, p)
        assert eta == round(math.log2(1 / p))
        assert params.bloom_fpr(m, n, eta) == pytest.approx(p, rel=0.15)
        # the printed formula without the divisor gives a filter too small
        m_printed = math.ceil(-n * math.log(p) / math.log(2))
        assert params.bloom_fpr(m_printed, n, eta) > 1.5 * p


def test_bloom_fpr_closed_form_small_cases():
    # one insertion, one hash: exactly 1/m of the bits set
    assert params.bloom_fpr(64, 1, 1) == pytest.approx(1 / 64)
    # two insertions, one hash: 1 - (1 - 1/m)^2
    assert params.bloom_fpr(100, 2, 1) == pytest.approx(1 - 0.99 ** 2)
    assert params.bloom_fpr(1000, 0, 3) == 0.0


def test_repetitions_is_the_smallest_meeting_lemma_4_2():
    for K, B, p, V, delta in [(1000, 50, 0.01, 1, 0.01), (100_000, 1000, 0.001, 5, 1e-3), (17618, 2000, 0.02, 10, 0.05)]:
        R = params.repetitions(K, B, p, V, delta)
        assert params.failure_bound(K, B, R, p, V) <= delta * (1 + 1e-9)
        if R > 1:
            assert params.failure_bound(K, B, R - 1, p, V) > delta
        # and R grows like log K - log delta (Theorem 4.3)
        R2 = params.repetitions(K * 100, B, p, V, delta)
        assert R2 > R


def test_cells_minimise_expected_query_time():
    for K, V, eta in [(1000, 1, 2), (100_000, 4, 2), (17618, 10, 4)]:
        B = params.cells(K, V, eta)
        assert B == round(math.sqrt(K * V / eta))
        t = lambda b: params.expected_query_time(K, b, 3, eta, V, 0.0)
        grid = range(max(1, B // 4), min(K, 4 * B) + 1)
        best = min(grid, key=t)
        assert abs(best - B) <= 1


def test_suggest_fits_the_library_limits():
    s = params.suggest(100_000, 2e6, p=0.01, V=2, delta=1e-3)
    assert 1 <= s.B <= params.MAX_B and 1 <= s.R <= params.MAX_R and s.R * s.eta <= params.MAX_RETA
    assert s.failure_bound <= 1e-3 * (1 + 1e-9) or s.notes
    assert s.bfu_fpr <= 0.01 * 1.2
    cfg = s.config()
    assert set(cfg) == {"K", "B", "R", "eta", "k", "m"}
    # R * eta over the limit: eta lowered and m raised so p still holds
    s2 = params.suggest(10 ** 6, 1e4, p=1e-6, V=50, delta=1e-9)
    assert s2.R * s2.eta <= params.MAX_RETA and s2.notes
    assert s2.bfu_fpr <= 1e-6 * (1 + 1e-6)


def test_suggested_size_gives_target_rate_on_a_built_index():
    # Sec. 5.1: size every BFU from the mean cardinality of a prefix
    # sample; the filters built with that size have false-positive rate
    # about p (measured as fill^eta on the oracle's filters, the rate of
    # a random absent term)
    K, k, p, ns = 256, 21, 0.02, 32
    sets = synth.genome_sets(41, K=K, n_ancestors=K, ancestor_len=2000, median_len=1500, min_len=1000,
                             max_len=2000)
    sample = sets.offsets[:ns + 1]       # the first ns sets
    codes = oracle.extract(sample, sets.chars[: int(sample[-1])], k)
    seg = np.repeat(np.arange(ns), np.diff(sample).astype(np.int64))
    distinct = [np.unique(codes[(seg == s) & (codes != oracle.NO_KMER)]).size for s in range(ns)]
    mean = params.mean_distinct_terms(codes, sample, invalid=oracle.NO_KMER)
    assert mean == pytest.approx(np.mean(distinct))
    s = params.suggest(K, mean, p=p, V=1, delta=0.01, B=8)
    o = oracle.OracleIndex(K, s.B, s.R, s.eta, k, s.m, 5)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 4)
    fill = o.fill_counts().astype(np.float64) / s.m
    rate = fill ** s.eta
    assert rate.mean() == pytest.approx(p, rel=0.35)
    assert rate.max() < 2 * p
