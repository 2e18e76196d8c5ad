"""Seeded synthetic workloads (genomes, k-mer queries, reads, request streams).

Stand-ins for the paper's ENA whole-genome data (Sec. 5.2): each set is one
genome, each term a 31-mer of an ACGT sequence.  Everything is drawn from a
Philox counter-based generator (Salmon et al., SC'11) keyed by a seed, so the
same seed yields the same bytes on every machine.  This module produces raw
bytes and integers only; it holds no encoding, hashing or indexing
arithmetic, and it serves the GPU path and the test oracle alike.

Every workload is a CSR of byte sequences: ``chars`` (uint8, concatenated),
``offsets`` (uint64, n+1) and, for sets, ``set_ids`` (uint32, n).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_LUT = np.frombuffer(b"ACGT", dtype=np.uint8)
SIGMA_LOGNORMAL = math.log(10.0) / 3.0   # a decade is three sigma


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


@dataclass
class SeqBatch:
    chars: np.ndarray                  # uint8
    offsets: np.ndarray                # uint64, n+1
    set_ids: np.ndarray | None = None  # uint32, n (sets only)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.offsets.size - 1

    def seq(self, i: int) -> bytes:
        return self.chars[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)


def _csr(parts: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    lens = np.array([p.size for p in parts], dtype=np.uint64)
    offsets = np.zeros(len(parts) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    chars = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return np.ascontiguousarray(chars, dtype=np.uint8), offsets


def random_bases(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random bases as base indices 0..3 (the 2-bit digits of
    uniform 64-bit words)."""
    words = rng.integers(0, 2**64, size=(n + 31) // 32, dtype=np.uint64)
    out = np.empty(((n + 31) // 32) * 32, np.uint8)
    w8 = words.view(np.uint8)                       # little-endian bytes, 4 digits each
    for d in range(4):
        out[d::4] = (w8 >> np.uint8(2 * d)) & np.uint8(3)
    return out[:n]


def substitute(rng: np.random.Generator, idx: np.ndarray, rate: float) -> np.ndarray:
    """Every position independently, with probability `rate`, becomes one of
    the other three bases, uniformly (a Bernoulli process drawn as geometric
    gaps)."""
    out = idx.copy()
    if rate <= 0 or out.size == 0:
        return out
    pos = _bernoulli_positions(rng, out.size, rate)
    out[pos] = (out[pos] + rng.integers(1, 4, size=pos.size, dtype=np.uint8)) & 3
    return out


def lognormal_lengths(rng, n, median, lo, hi, sigma=SIGMA_LOGNORMAL) -> np.ndarray:
    x = np.exp(rng.normal(math.log(median), sigma, size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def to_bytes(idx: np.ndarray) -> np.ndarray:
    return _LUT[idx]


# --------------------------------------------------------------------- sets

def genome_sets(seed: int, K: int, n_ancestors: int, ancestor_len: int, *,
                sub_rate: float = 0.01, median_len: int | None = None,
                min_len: int | None = None, max_len: int | None = None) -> SeqBatch:
    """K genomes: set i is a window of ancestor (i mod n_ancestors) with
    independent substitutions.  With median_len None every set is the whole
    ancestor; otherwise the window length is lognormal (clipped).  The
    ancestors are drawn at once, the windows copied into place, and the
    substitutions drawn as one Bernoulli process over all genomes (the same
    law as per genome: every base independently)."""
    rng = rng_for(seed)
    anc = _LUT[random_bases(rng, n_ancestors * ancestor_len)].reshape(n_ancestors, ancestor_len)
    if median_len is None:
        lens = np.full(K, ancestor_len, dtype=np.int64)
    else:
        lens = lognormal_lengths(rng, K, median_len, min_len, min(max_len, ancestor_len))
    starts = (rng.random(K) * (ancestor_len - lens + 1)).astype(np.int64)
    offsets = np.zeros(K + 1, dtype=np.uint64)
    np.cumsum(lens.astype(np.uint64), out=offsets[1:])
    chars = np.empty(int(offsets[-1]), dtype=np.uint8)   # filled in place: no second copy of the genomes
    for i in range(K):
        o, L, st = int(offsets[i]), int(lens[i]), int(starts[i])
        chars[o:o + L] = anc[i % n_ancestors, st:st + L]
    del anc
    _substitute_bytes(rng, chars, sub_rate)
    return SeqBatch(chars, offsets, np.arange(K, dtype=np.uint32),
                    meta=dict(K=K, n_ancestors=n_ancestors, ancestor_len=ancestor_len,
                              sub_rate=sub_rate, median_len=median_len))


def _substitute_bytes(rng: np.random.Generator, chars: np.ndarray, rate: float, chunk: int = 1 << 28) -> None:
    """In place, on ACGT bytes: every position independently, with
    probability `rate`, becomes one of the other three bases, uniformly
    (drawn chunk by chunk so that memory stays bounded)."""
    if rate <= 0:
        return
    back = np.zeros(256, np.uint8)
    back[_LUT] = np.arange(4, dtype=np.uint8)
    for a in range(0, chars.size, chunk):
        seg = chars[a:a + chunk]
        pos = _bernoulli_positions(rng, seg.size, rate)
        seg[pos] = _LUT[(back[seg[pos]] + rng.integers(1, 4, size=pos.size, dtype=np.uint8)) & 3]


def _bernoulli_positions(rng: np.random.Generator, L: int, rate: float) -> np.ndarray:
    """Positions in [0, L) of a Bernoulli(rate) process, drawn as geometric gaps."""
    if L == 0:
        return np.zeros(0, np.int64)
    mean = L * rate
    draw = int(mean + 10 * math.sqrt(mean) + 16)
    pos = np.cumsum(rng.geometric(rate, size=draw)) - 1
    while pos[-1] < L:
        more = np.cumsum(rng.geometric(rate, size=draw)) + pos[-1]
        pos = np.concatenate([pos, more])
    return pos[pos < L]


# ------------------------------------------------------------------ queries

def kmer_queries(seed: int, sets: SeqBatch, n: int, k: int, present_frac: float = 0.5) -> SeqBatch:
    """n single k-mer queries as k-byte sequences: the first round(n *
    present_frac) are windows at a uniform (set, position) of the inserted
    genomes, the rest uniform random ACGT strings.  Order is shuffled; the
    'present' mask and 'source_set' (the sequence a present query was cut
    from, -1 for random ones) are kept in meta."""
    rng = rng_for(seed)
    n_pres = int(round(n * present_frac))
    lens = sets.lengths().astype(np.int64)
    ok = np.nonzero(lens >= k)[0]
    which = ok[rng.integers(0, ok.size, size=n_pres)]
    starts = sets.offsets[which].astype(np.int64) + (rng.random(n_pres) * (lens[which] - k + 1)).astype(np.int64)
    out = np.empty((n, k), dtype=np.uint8)
    step = 1 << 20
    for lo in range(0, n_pres, step):
        hi = min(n_pres, lo + step)
        out[lo:hi] = sets.chars[starts[lo:hi, None] + np.arange(k)[None, :]]
    out[n_pres:] = to_bytes(random_bases(rng, (n - n_pres) * k)).reshape(n - n_pres, k)
    perm = rng.permutation(n)
    out = out[perm]
    present = np.zeros(n, dtype=bool)
    present[:n_pres] = True
    present = present[perm]
    src = np.full(n, -1, dtype=np.int64)
    src[:n_pres] = which
    src = src[perm]
    offsets = np.arange(n + 1, dtype=np.uint64) * np.uint64(k)
    return SeqBatch(out.reshape(-1), offsets, None, meta=dict(present=present, source_set=src, k=k))


def reads(seed: int, sets: SeqBatch, n: int, *, median_len: int, min_len: int, max_len: int,
          substr_frac: float, read_sub_rate: float = 0.0, lengths: np.ndarray | None = None) -> SeqBatch:
    """n reads.  A fraction substr_frac are substrings of a uniformly chosen
    set genome (cut to the genome's length), optionally with further
    substitutions; the rest are uniform random ACGT.  Lengths are lognormal
    (clipped) unless given.  meta['source_set']: the genome of each
    substring read, -1 for random reads."""
    rng = rng_for(seed)
    if lengths is None:
        lengths = lognormal_lengths(rng, n, median_len, min_len, max_len)
    lengths = np.asarray(lengths, np.int64).copy()
    kind = rng.random(n) < substr_frac
    glens = sets.lengths().astype(np.int64)
    n_sub = int(kind.sum())
    g = rng.integers(0, sets.n, size=n_sub)
    sub = np.nonzero(kind)[0]
    lengths[sub] = np.minimum(lengths[sub], glens[g])
    st = sets.offsets[g].astype(np.int64) + (rng.random(n_sub) * (glens[g] - lengths[sub] + 1)).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths.astype(np.uint64), out=offsets[1:])
    chars = np.empty(int(offsets[-1]), dtype=np.uint8)
    # substring reads: one gather of every byte (start of the read's source
    # + position in the read), in chunks of reads
    o64 = offsets.astype(np.int64)
    for a in range(0, n_sub, 1 << 18):
        q = sub[a:a + (1 << 18)]
        L = lengths[q]
        dst = np.repeat(o64[q], L) + _ranges(L)
        src = np.repeat(st[a:a + (1 << 18)], L) + _ranges(L)
        chars[dst] = sets.chars[src]
        if read_sub_rate > 0:
            seg = chars[dst]
            _substitute_bytes(rng, seg, read_sub_rate)
            chars[dst] = seg
    rnd = np.nonzero(~kind)[0]
    for a in range(0, rnd.size, 1 << 18):
        q = rnd[a:a + (1 << 18)]
        L = lengths[q]
        dst = np.repeat(o64[q], L) + _ranges(L)
        chars[dst] = _LUT[random_bases(rng, int(L.sum()))]
    src_set = np.full(n, -1, dtype=np.int64)
    src_set[sub] = g
    return SeqBatch(chars, offsets, None, meta=dict(source_set=src_set))


def _ranges(L: np.ndarray) -> np.ndarray:
    """Concatenation of arange(l) for every l in L."""
    L = np.asarray(L, np.int64)
    total = int(L.sum())
    if total == 0:
        return np.zeros(0, np.int64)
    starts = np.cumsum(L) - L
    return np.arange(total, dtype=np.int64) - np.repeat(starts, L)


# ---------------------------------------------------------------- documents

@dataclass
class KeyBatch:
    """CSR of 64-bit keys: keys of item i are keys[offsets[i] .. offsets[i+1])."""
    keys: np.ndarray                   # uint64
    offsets: np.ndarray                # uint64, n+1
    set_ids: np.ndarray | None = None  # uint32, n (sets only)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.offsets.size - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)


def zipf_ranks(rng: np.random.Generator, n: int, vocab: int, s: float) -> np.ndarray:
    """n word ranks in [0, vocab), rank r drawn with probability proportional
    to (r+1)^-s (a Zipf law truncated to the vocabulary)."""
    cdf = np.cumsum(np.arange(1, vocab + 1, dtype=np.float64) ** -s)
    cdf /= cdf[-1]
    out = np.empty(n, np.int64)
    for a in range(0, n, 1 << 24):
        b = min(n, a + (1 << 24))
        out[a:b] = np.minimum(np.searchsorted(cdf, rng.random(b - a)), vocab - 1)
    return out


def documents(seed: int, K: int, *, vocab: int, median_len: int, min_len: int, max_len: int,
              zipf_s: float = 1.07) -> KeyBatch:
    """K documents as sets of word keys, a stand-in for the word-unigram
    corpora of Sec. 5.3: a vocabulary of `vocab` distinct random 64-bit keys
    (the word -> key map is the caller's, so words are just keys here);
    document i has a log-normal number of tokens in [min_len, max_len] drawn
    from a Zipf law over the vocabulary ranks, and keeps its distinct words.
    meta: the vocabulary (rank order) and the Zipf exponent."""
    rng = rng_for(seed)
    words = np.unique(rng.integers(0, 2**64, size=vocab + vocab // 64 + 64, dtype=np.uint64))
    words = rng.permutation(words)[:vocab]
    lens = lognormal_lengths(rng, K, median_len, min_len, max_len)
    ranks = zipf_ranks(rng, int(lens.sum()), vocab, zipf_s)
    # distinct (document, rank) pairs, in document order then rank order
    pairs = np.unique(np.repeat(np.arange(K, dtype=np.int64), lens) * vocab + ranks)
    doc = pairs // vocab
    offsets = np.zeros(K + 1, np.uint64)
    np.cumsum(np.bincount(doc, minlength=K), out=offsets[1:])
    keys = np.ascontiguousarray(words[pairs % vocab], np.uint64)
    return KeyBatch(keys, offsets, np.arange(K, dtype=np.uint32), dict(vocab=words, zipf_s=zipf_s))


def word_queries(seed: int, docs: KeyBatch, n: int, present_frac: float = 0.5) -> np.ndarray:
    """n single-word queries (uint64 keys): round(n * present_frac) vocabulary
    words drawn by the same Zipf law as the text (popular words are asked
    for more often, as in a query log), the rest random keys outside the
    vocabulary.  Shuffled."""
    rng = rng_for(seed)
    vocab = docs.meta["vocab"]
    n_in = int(round(n * present_frac))
    hit = vocab[zipf_ranks(rng, n_in, vocab.size, docs.meta["zipf_s"])]
    miss = rng.integers(0, 2**64, size=n - n_in, dtype=np.uint64)
    miss = miss[~np.isin(miss, vocab)]
    q = np.concatenate([hit, miss, rng.integers(0, 2**64, size=n - n_in - miss.size, dtype=np.uint64)])
    return rng.permutation(q).astype(np.uint64)


def word_sets(seed: int, docs: KeyBatch, n: int, min_words: int = 1, max_words: int = 4,
              from_doc_frac: float = 0.5) -> KeyBatch:
    """n multi-word queries (term sets, Sec. 3.2.1 applied to words): each
    has a uniform number of words in [min_words, max_words]; a share
    from_doc_frac of them take their words from one random document (so it
    answers them), the rest draw vocabulary words by the Zipf law of the
    text.  Words may repeat within a query."""
    rng = rng_for(seed)
    vocab = docs.meta["vocab"]
    lens = rng.integers(min_words, max_words + 1, size=n)
    offsets = np.zeros(n + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    owner = np.repeat(np.arange(n), lens)
    dl = docs.lengths().astype(np.int64)
    nonempty = np.nonzero(dl > 0)[0]
    from_doc = (rng.random(n) < from_doc_frac) & (nonempty.size > 0)
    doc = nonempty[rng.integers(0, max(1, nonempty.size), size=n)] if nonempty.size else np.zeros(n, np.int64)
    kd = from_doc[owner]
    keys = vocab[zipf_ranks(rng, owner.size, vocab.size, docs.meta["zipf_s"])].astype(np.uint64)
    dk = doc[owner[kd]]
    pos = docs.offsets[dk].astype(np.int64) + (rng.random(dk.size) * dl[dk]).astype(np.int64)
    keys[kd] = docs.keys[pos]
    return KeyBatch(keys, offsets)


# ---------------------------------------------------------------- workloads

def config_tiny(seed: int = 1001) -> SeqBatch:
    """64 sets, each one of 8 random 5 000 bp ancestors with 1% substitutions."""
    return genome_sets(seed, K=64, n_ancestors=8, ancestor_len=5000)


def config_mid(seed: int = 1002) -> SeqBatch:
    """1 000 sets: lognormal windows (median 200 kbp, 20 kbp - 2 Mbp) of 50
    random 2 Mbp ancestors, 1% substitutions (about 2.7e8 bases)."""
    return genome_sets(seed, K=1000, n_ancestors=50, ancestor_len=2_000_000,
                       median_len=200_000, min_len=20_000, max_len=2_000_000)


def config_batched_reads(sets: SeqBatch, n: int = 100_000, seed: int = 3003) -> SeqBatch:
    """Reads of lognormal length (median 1 000, 100 - 10 000 bp): 70% exact
    substrings of a set genome, 30% random."""
    return reads(seed, sets, n, median_len=1000, min_len=100, max_len=10_000, substr_frac=0.7)


def config_served(seed: int = 1004) -> SeqBatch:
    """10 000 sets: lognormal windows (median 500 kbp, 50 kbp - 5 Mbp) of 500
    random 5 Mbp ancestors, 1% substitutions (about 6.7e9 bases)."""
    return genome_sets(seed, K=10_000, n_ancestors=500, ancestor_len=5_000_000,
                       median_len=500_000, min_len=50_000, max_len=5_000_000)


def config_large(seed: int = 1005) -> SeqBatch:
    """100 000 sets: lognormal windows (median 100 kbp, 10 kbp - 1 Mbp) of
    5 000 random 1 Mbp ancestors, 1% substitutions (about 1.3e10 bases)."""
    return genome_sets(seed, K=100_000, n_ancestors=5000, ancestor_len=1_000_000,
                       median_len=100_000, min_len=10_000, max_len=1_000_000)


def served_requests(seed: int, sets: SeqBatch, n_requests: int, *, min_reads: int = 1, max_reads: int = 64,
                    min_len: int = 150, max_len: int = 5000, substr_frac: float = 0.7) -> SeqBatch:
    """n_requests requests of U{min_reads..max_reads} reads each, read lengths
    log-uniform in [min_len, max_len], 70% exact substrings of a set genome
    and 30% random.  All reads in one batch; meta['request_offsets'] (n+1)
    delimits the requests' reads."""
    rng = rng_for(seed)
    per = rng.integers(min_reads, max_reads + 1, size=n_requests)
    n = int(per.sum())
    lengths = np.rint(np.exp(rng.uniform(math.log(min_len), math.log(max_len), size=n))).astype(np.int64)
    batch = reads(seed + 1, sets, n, median_len=0, min_len=min_len, max_len=max_len,
                  substr_frac=substr_frac, lengths=lengths)
    ro = np.zeros(n_requests + 1, dtype=np.int64)
    np.cumsum(per, out=ro[1:])
    batch.meta["request_offsets"] = ro
    return batch


def request(batch: SeqBatch, r: int) -> tuple[np.ndarray, np.ndarray]:
    """(offsets rebased to 0, bytes) of request r of a served_requests batch."""
    ro = batch.meta["request_offsets"]
    a, b = int(ro[r]), int(ro[r + 1])
    off = batch.offsets[a:b + 1]
    return (off - off[0]).astype(np.uint64), batch.chars[int(off[0]):int(off[-1])]


def poisson_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    """n arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = rng_for(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# Index parameters of the workloads: K sets, B cells, R repetitions, m bits per
# cell, eta hashes, k-mer length.
INDEX_TINY = dict(K=64, B=8, R=3, m=1 << 18, eta=2, k=31)
INDEX_MID = dict(K=1000, B=50, R=4, m=1 << 28, eta=2, k=31)
INDEX_SERVED = dict(K=10_000, B=200, R=5, m=1 << 29, eta=2, k=31)
INDEX_LARGE = dict(K=100_000, B=1000, R=6, m=1 << 27, eta=2, k=31)
# the word-unigram index of Sec. 5.3 (the Wikipedia sample's K, B, R and
# filter size); eta is this workload's choice
INDEX_WIKI = dict(K=17_618, B=2000, R=2, m=200_000, eta=4, k=31)


def config_wiki(seed: int = 1006) -> KeyBatch:
    """17 618 documents over a 500 000-word vocabulary, about 1 500 tokens
    each (median; 50 to 20 000), Zipf exponent 1.07."""
    return documents(seed, 17_618, vocab=500_000, median_len=1500, min_len=50, max_len=20_000)
