"""Parameter helper: choosing m, eta, B and R for a RAMBO index (host only).

Each rule is the paper's, in its own notation:

* Bloom filter of n insertions at false-positive rate p (Sec. 2):
  eta = -log2 p hashes and m = -n ln p / (ln 2)^2 bits, the standard optimum
  (the printed size formula lacks the (ln 2)^2 divisor; with it,
  (1 - e^{-eta n / m})^eta = p at eta = -log2 p).  The false-positive rate
  of a given filter is (1 - (1 - 1/m)^{eta n})^eta.
* A BFU holds the union of the K/B sets of its cell (Sec. 3), so its
  insertions are at most K/B times the mean set cardinality; Sec. 5.1 sizes
  every BFU from the mean cardinality of a small prefix sample of the sets.
* Lemma 4.2 bounds the probability of a wrong membership for any of the K
  sets by delta <= K (1 - (1 - p)(1 - 1/B)^V)^R for a term in at most V sets;
  the smallest R meeting a target delta follows, R = O(log K - log delta)
  (Theorem 4.3).
* The expected query time B R eta + (K / B)(V + B p) R (Sec. 4.2) is least at
  B = sqrt(K V / eta).

suggest() combines them into a configuration that rambo_create accepts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

MAX_B = 4096      # limits of the library (include/rambo.h)
MAX_R = 16
MAX_RETA = 32


def bloom_hashes(p: float) -> int:
    """eta = -log2 p, rounded, at least 1 (Sec. 2)."""
    if not 0.0 < p < 1.0:
        raise ValueError("p must lie in (0, 1)")
    return max(1, round(-math.log2(p)))


def bloom_bits(n: float, p: float) -> int:
    """m = -n ln p / (ln 2)^2 bits for n insertions at rate p (Sec. 2, with
    the (ln 2)^2 divisor), at least 64."""
    if n < 0 or not 0.0 < p < 1.0:
        raise ValueError("need n >= 0 and p in (0, 1)")
    return max(64, math.ceil(-n * math.log(p) / math.log(2.0) ** 2))


def bloom_fpr(m: int, n: float, eta: int) -> float:
    """(1 - (1 - 1/m)^{eta n})^eta (Sec. 2)."""
    return (1.0 - (1.0 - 1.0 / m) ** (eta * n)) ** eta


def bfu_insertions(mean_set_terms: float, K: int, B: int) -> float:
    """Insertions into one BFU: the K/B sets of a cell, each with the mean
    cardinality (an upper bound: terms shared by sets of one cell count once
    in the filter)."""
    return mean_set_terms * K / B


def mean_distinct_terms(codes, offsets, invalid=None) -> float:
    """Mean number of distinct terms per set of a prefix sample (Sec. 5.1):
    codes[offsets[s] .. offsets[s+1]) are the terms of sampled set s (for
    example the k-mer codes Rambo.extract_kmers gives for the sample's
    bytes, copied to the host); entries equal to `invalid` are skipped."""
    import numpy as np
    codes = np.asarray(codes)
    offsets = np.asarray(offsets, dtype=np.int64)
    counts = []
    for s in range(offsets.size - 1):
        c = codes[offsets[s]:offsets[s + 1]]
        if invalid is not None:
            c = c[c != invalid]
        counts.append(np.unique(c).size)
    return float(np.mean(counts)) if counts else 0.0


def failure_bound(K: int, B: int, R: int, p: float, V: int) -> float:
    """Lemma 4.2: K (1 - (1 - p)(1 - 1/B)^V)^R."""
    return K * (1.0 - (1.0 - p) * (1.0 - 1.0 / B) ** V) ** R


def repetitions(K: int, B: int, p: float, V: int, delta: float) -> int:
    """The smallest R with failure_bound(K, B, R, p, V) <= delta."""
    if not 0.0 < delta < 1.0:
        raise ValueError("delta must lie in (0, 1)")
    q = 1.0 - (1.0 - p) * (1.0 - 1.0 / B) ** V
    if q <= 0.0:
        return 1
    if q >= 1.0:
        raise ValueError("no R reaches delta: every cell is positive (B = 1 or p = 1)")
    return max(1, math.ceil((math.log(K) - math.log(delta)) / -math.log(q) - 1e-12))


def expected_query_time(K: int, B: int, R: int, eta: int, V: int, p: float) -> float:
    """B R eta + (K / B)(V + B p) R (expected query time, Sec. 4.2)."""
    return B * R * eta + (K / B) * (V + B * p) * R


def cells(K: int, V: int, eta: int) -> int:
    """B = sqrt(K V / eta), rounded, within [1, min(K, MAX_B)]."""
    return int(min(max(1, round(math.sqrt(K * V / eta))), K, MAX_B))


@dataclass
class Suggestion:
    K: int
    B: int
    R: int
    eta: int
    m: int
    bfu_insertions: float
    bfu_fpr: float           # predicted p of one BFU
    failure_bound: float     # Lemma 4.2 at the chosen B, R, p
    index_bytes: int         # R * m * S / 8 with S = max(8, next_pow2(B))
    notes: list

    def config(self, k: int = 31) -> dict:
        """Keyword arguments of Rambo(...) (seed excluded)."""
        return dict(K=self.K, B=self.B, R=self.R, eta=self.eta, k=k, m=self.m)


def _row_bits(B: int) -> int:
    s = 8
    while s < B:
        s *= 2
    return s


def suggest(K: int, mean_set_terms: float, *, p: float = 0.01, V: int = 1, delta: float = 0.01,
            B: int | None = None, eta: int | None = None) -> Suggestion:
    """A configuration for K sets of mean cardinality mean_set_terms (from a
    prefix sample, Sec. 5.1): eta from p, B from the query-time optimum
    (or given), m for the BFU's insertions at p, R from Lemma 4.2 for terms
    in at most V sets and failure probability delta.  Values clamped to the
    library's limits are listed in notes."""
    notes = []
    eta = bloom_hashes(p) if eta is None else eta
    B = cells(K, V, eta) if B is None else B
    if not 1 <= B <= min(K, MAX_B):
        raise ValueError("B out of range")
    n = bfu_insertions(mean_set_terms, K, B)
    m = bloom_bits(n, p)
    fpr = bloom_fpr(m, n, eta)
    R = repetitions(K, B, fpr, V, delta)
    if R > MAX_R:
        notes.append("R = %d clamped to %d" % (R, MAX_R))
        R = MAX_R
    if R * eta > MAX_RETA:
        e2 = max(1, MAX_RETA // R)
        notes.append("eta = %d lowered to %d (R * eta <= %d); m raised to keep p" % (eta, e2, MAX_RETA))
        eta = e2
        m = _bits_for_rate(n, eta, p)
        fpr = bloom_fpr(m, n, eta)
    return Suggestion(K=K, B=B, R=R, eta=eta, m=m, bfu_insertions=n, bfu_fpr=fpr,
                      failure_bound=failure_bound(K, B, R, fpr, V),
                      index_bytes=R * m * _row_bits(B) // 8, notes=notes)


def _bits_for_rate(n: float, eta: int, p: float) -> int:
    """Smallest m (>= 64) with bloom_fpr(m, n, eta) <= p for a fixed eta:
    m = 1 / (1 - (1 - p^{1/eta})^{1/(eta n)})."""
    if n <= 0:
        return 64
    x = 1.0 - p ** (1.0 / eta)              # (1 - 1/m)^{eta n} must be >= x
    return max(64, math.ceil(1.0 / -math.expm1(math.log(x) / (eta * n))))
