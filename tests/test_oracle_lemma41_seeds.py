"""Unconditional Lemma 4.1 (Sec. 4.1) over many seeds: for each of 32 seeds
(each draws its own partition, hash multipliers, keys and set IDs) the
oracle indexes N sets of L random keys, and the false-positive rate of
random queries (V = 0) and of keys planted in V sets is measured over those
sets; the mean over seeds must lie within 3 standard errors (the spread
across seeds) of Lemma 4.1 with the Bloom-filter rate p averaged over the
partition (oracle.fpr).  Over 1e6 random queries in all.

The lemma's proof takes every set's cell as uniform and independent of the
others'.  The partition hash is the 2-universal affine map, which on
consecutive IDs 0..N-1 spreads the sets far more evenly than independent
throws would (cell loads within one or two of the mean); so the N sets get
random distinct IDs from [0, K) with K >> N, on which the affine map behaves
like independent throws, and only those sets are counted."""
import math

import numpy as np
import pytest

import oracle
from oracle import fpr

N, K, B, R, ETA, M, L = 200, 8192, 20, 3, 2, 1 << 14, 500
SEEDS = 32
RANDOM_PER_SEED = 32_000
PLANTED = {1: 2000, 4: 2000, 16: 2000}   # V -> planted queries per seed


def _fp_rate(masks, holders, ids):
    """False positives over the indexed sets ids, per (query, set not holding it)."""
    bits = np.unpackbits(masks.view(np.uint8), axis=1, bitorder="little")[:, ids].astype(bool)
    fp = bits.sum(axis=1) - np.array([len(h) for h in holders])
    for t, h in enumerate(holders):   # no false negatives (h: positions in ids)
        assert bits[t, list(h)].all()
    return float(fp.sum()) / float(sum(N - len(h) for h in holders))


def _one_seed(seed):
    rng = np.random.default_rng(1000 + seed)
    o = oracle.OracleIndex(K, B, R, ETA, 31, M, seed=7000 + seed, flags=oracle.FLAG_RAW_KEYS)
    ids = np.sort(rng.choice(K, size=N, replace=False)).astype(np.uint32)
    keys = rng.integers(0, 1 << 62, size=N * L, dtype=np.uint64)
    offsets = np.arange(N + 1, dtype=np.uint64) * np.uint64(L)
    assert o.insert_kmers(ids, offsets, keys, nthreads=4) == 0
    # random queries: V = 0 (a 62-bit collision with an inserted key is ~1e-13)
    q = rng.integers(0, 1 << 62, size=RANDOM_PER_SEED, dtype=np.uint64)
    out = {0: _fp_rate(o.query_kmers(q, nthreads=4), [()] * q.size, ids)}
    # planted: a fresh key inserted into V random sets of the N, then queried
    for V, n in PLANTED.items():
        codes = rng.integers(0, 1 << 62, size=n, dtype=np.uint64)
        holders = [tuple(int(i) for i in rng.choice(N, size=V, replace=False)) for _ in range(n)]
        who = np.array([i for h in holders for i in h], np.int64)
        ks = np.repeat(codes, V)
        order = np.argsort(who, kind="stable")
        who, ks = who[order], ks[order]
        off = np.zeros(N + 1, np.uint64)
        np.cumsum(np.bincount(who, minlength=N), out=off[1:])
        assert o.insert_kmers(ids, off, ks, nthreads=4) == 0
        out[V] = _fp_rate(o.query_kmers(codes, nthreads=4), holders, ids)
    o.close()
    return out


def keys_in_cell(s, V):
    """Distinct keys of a cell holding s sets when the queries of multiplicity
    V are asked: L of each set, and one key of every planted query so far
    that has a holder among them (holders of a query are V distinct sets
    drawn from the N, so one lands in the cell with probability
    1 - C(N - s, v) / C(N, v)); the query asked is not in the cell."""
    keys = s * L
    for v, n in PLANTED.items():
        if v <= V:
            keys += (n - (1 if v == V else 0)) * (1.0 - math.comb(N - s, v) / math.comb(N, v))
    return keys


@pytest.fixture(scope="module")
def sweep():
    runs = [_one_seed(s) for s in range(SEEDS)]
    return {V: np.array([r[V] for r in runs]) for V in [0] + list(PLANTED)}


@pytest.mark.parametrize("V", [0] + list(PLANTED))
def test_unconditional_lemma41_over_seeds(sweep, V):
    obs = sweep[V]
    pred = fpr.lemma41_over_partitions(N, B, V, R, lambda s: keys_in_cell(s, V), M, ETA)
    se = obs.std(ddof=1) / math.sqrt(obs.size)
    z = (obs.mean() - pred) / se
    print("V=%d: observed %.5f +- %.5f over %d seeds, Lemma 4.1 %.5f, z %.2f" % (V, obs.mean(), se, obs.size, pred, z))
    assert abs(z) < 3.0, (V, obs.mean(), pred, se, z)
    assert RANDOM_PER_SEED * SEEDS >= 1_000_000


def test_partition_average_special_cases():
    # B = 1: every set shares the one cell, so p is Sec. 2's rate for N*L keys
    assert fpr.cell_fpr_over_partitions(N, 1, 0, L, M, ETA) == pytest.approx(fpr.bf_fpr(N * L, M, ETA), rel=1e-12)
    # one set: its cell holds its own L keys
    assert fpr.cell_fpr_over_partitions(1, B, 0, L, M, ETA) == pytest.approx(fpr.bf_fpr(L, M, ETA), rel=1e-12)
    # the average lies between the rates of the emptiest and fullest cells and
    # above the rate of the mean load (the rate is convex in the load here)
    p = fpr.cell_fpr_over_partitions(N, B, 0, L, M, ETA)
    assert fpr.bf_fpr(L, M, ETA) < fpr.bf_fpr((1 + (N - 1) / B) * L, M, ETA) < p < fpr.bf_fpr(N * L, M, ETA)
    # against the binomial mixture sampled directly
    rng = np.random.default_rng(9)
    n = rng.binomial(N - 1, 1.0 / B, size=2_000_000)
    mc = np.mean(fpr.bf_fpr(1.0, M, ETA) * 0 + (-np.expm1(ETA * (1 + n) * L * math.log1p(-1.0 / M))) ** ETA)
    assert p == pytest.approx(mc, rel=2e-3)


def test_consecutive_ids_spread_evenly():
    # why the sweep uses random IDs: on IDs 0..N-1 the affine partition's
    # loads vary far less than independent throws' (variance N/B (1 - 1/B))
    o = oracle.OracleIndex(N, B, R, ETA, 31, M, seed=11, flags=oracle.FLAG_RAW_KEYS)
    loads = np.array([np.bincount(row, minlength=B) for row in o.phi()])
    o.close()
    assert loads.var() < 0.5 * (N / B) * (1 - 1 / B)
