"""False-positive predictions for the oracle's validation (test infrastructure).

* Sec. 2: a Bloom filter of m bits holding n keys with eta hashes has every
  bit set with probability 1 - (1 - 1/m)^(eta n), and false-positive rate
  p = (1 - (1 - 1/m)^(eta n))^eta.
* Lemma 4.1: a query q held by V sets is reported for a set that does not
  hold it with probability (p (1 - 1/B)^V + 1 - (1 - 1/B)^V)^R.
* The same lemma with p averaged over random partitions, for sets of equal
  size (the unconditional form, compared with the mean over many seeds).
* The same lemma conditioned on the realised partition and cell fills (the
  quantity its proof averages): in repetition r, set i's cell passes for
  sure when it also holds one of q's true sets, and otherwise passes with
  that cell's own Bloom-filter false-positive rate; repetitions multiply.

All arithmetic is float64.
"""
from __future__ import annotations

import math

import numpy as np


def bf_fill_expected(n: float, m: int, eta: int) -> float:
    """Expected fraction of set bits (Sec. 2)."""
    return 1.0 - (1.0 - 1.0 / m) ** (eta * n)


def bf_fpr(n: float, m: int, eta: int) -> float:
    """Bloom-filter false-positive rate p (Sec. 2)."""
    return bf_fill_expected(n, m, eta) ** eta


def occupancy_zero_bits_moments(throws: int, m: int):
    """Mean and variance of the number of zero bits after `throws` uniform,
    independent bit positions are set in an m-bit array (classical occupancy:
    E = m q1^N, Var = m q1^N + m(m-1) q2^N - m^2 q1^(2N), q1 = 1-1/m,
    q2 = 1-2/m)."""
    N = float(throws)
    l1 = N * math.log1p(-1.0 / m)
    l2 = N * math.log1p(-2.0 / m)
    e = m * math.exp(l1)
    var = m * math.exp(l1) + m * (m - 1) * math.exp(l2) - (m * m) * math.exp(2 * l1)
    return e, max(var, 0.0)


def lemma41(p: float, B: int, V: int, R: int) -> float:
    """Lemma 4.1: per-set false-positive probability."""
    miss = (1.0 - 1.0 / B) ** V
    return (p * miss + 1.0 - miss) ** R


def cell_fpr_over_partitions(K: int, B: int, V: int, keys_in_cell, m: int, eta: int) -> float:
    """The Bloom-filter false-positive rate p of the cell that holds a set
    which does not hold the query, averaged over the random partition (the
    p of Lemma 4.1 when the V holders of the query lie in other cells):
    besides the set itself, each of the other K - 1 - V sets falls into its
    cell with probability 1/B, so the cell holds s = 1 + n sets with
    n ~ Binomial(K - 1 - V, 1/B); keys_in_cell(s) is the number of distinct
    keys such a cell holds (a number: that many keys per set), and a cell of
    N keys has p = (1 - (1 - 1/m)^(eta N))^eta (Sec. 2)."""
    from scipy.stats import binom
    n_other = K - 1 - V
    n = np.arange(n_other + 1, dtype=np.float64)
    pmf = binom.pmf(n, n_other, 1.0 / B)
    if callable(keys_in_cell):
        keys = np.array([float(keys_in_cell(int(x))) for x in 1 + n])
    else:
        keys = (1.0 + n) * float(keys_in_cell)
    fill = -np.expm1(eta * keys * math.log1p(-1.0 / m))
    return float(np.sum(pmf * fill ** eta))


def lemma41_over_partitions(K: int, B: int, V: int, R: int, keys_in_cell, m: int, eta: int) -> float:
    """Lemma 4.1 with p averaged over the partition as above (repetitions
    draw independent partitions, so the per-repetition pass probabilities
    multiply)."""
    return lemma41(cell_fpr_over_partitions(K, B, V, keys_in_cell, m, eta), B, V, R)


def lemma42_bound(p: float, B: int, V: int, R: int, K: int) -> float:
    """Lemma 4.2: union bound on the probability of any wrong set."""
    return K * (1.0 - (1.0 - p) * (1.0 - 1.0 / B) ** V) ** R


def cell_fpr(fill_counts: np.ndarray, m: int, eta: int) -> np.ndarray:
    """Per-cell false-positive rate from its measured fill: fill^eta."""
    return (np.asarray(fill_counts, dtype=np.float64) / m) ** eta


def report_probability(phi: np.ndarray, pcell: np.ndarray, truth) -> np.ndarray:
    """P(set i is reported) for every i, conditioned on the partition phi
    (R x K), per-cell false-positive rates pcell (R x B) and the true holder
    sets `truth` of the query.  True holders get probability 1."""
    R, K = phi.shape
    truth = list(truth)
    prob = np.ones(K, dtype=np.float64)
    for r in range(R):
        hit = np.zeros(pcell.shape[1], dtype=bool)
        for j in truth:
            hit[phi[r, j]] = True
        cells = phi[r]
        prob *= np.where(hit[cells], 1.0, pcell[r, cells])
    return prob


def fpr_gate(observed_fp: np.ndarray, expected_fp: np.ndarray, negatives: np.ndarray):
    """Compare observed and predicted false positives over independent queries.

    observed_fp[q]: false positives reported for query q; expected_fp[q]: the
    prediction; negatives[q]: number of sets that do not hold q.  Queries are
    independent given the index, so the standard error of the total comes from
    the per-query residuals.  Returns (observed FPR, predicted FPR, z)."""
    obs = np.asarray(observed_fp, dtype=np.float64)
    exp = np.asarray(expected_fp, dtype=np.float64)
    neg = float(np.sum(negatives))
    d = obs - exp
    n = d.size
    se = math.sqrt(max(np.var(d, ddof=1), 1e-300) * n) if n > 1 else float("inf")
    z = float(np.sum(d)) / se if se > 0 else 0.0
    return float(obs.sum() / neg), float(exp.sum() / neg), z
