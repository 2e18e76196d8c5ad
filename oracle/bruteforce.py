"""Exact multiple-set-membership answers by brute force (test infrastructure).

The MSMT problem (Sec. 1): given sets S_1..S_K of terms and a query q, return
exactly {i : q in S_i}.  Here the terms are canonical k-mers (Sec. 5.2), and
they are handled as *strings*: the canonical form of a window is the smaller
of the window and its reverse complement in the lexicographic order
A < C < G < T, which is the same order as the integer codes the index uses.
Nothing here shares code with the oracle's integer encoding, so agreement
between the two pins both.
"""
from __future__ import annotations

_COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")
_DIGITS = bytes.maketrans(b"ACGT", b"0123")
_BASES = frozenset(b"ACGT")


def revcomp_str(w: bytes) -> bytes:
    return w.translate(_COMP)[::-1]


def canonical_str(w: bytes) -> bytes:
    w = w.upper()
    rc = revcomp_str(w)
    return w if w <= rc else rc


def code_of_str(w: bytes) -> int:
    """Integer code of an ACGT string through Python's base-4 int parser."""
    return int(w.upper().translate(_DIGITS), 4)


def kmers_of(seq: bytes, k: int):
    """Canonical k-mer strings of every window made only of ACGTacgt."""
    up = seq.upper()
    out = []
    for t in range(len(up) - k + 1):
        w = up[t:t + k]
        if all(c in _BASES for c in w):
            out.append(canonical_str(w))
    return out


class ExactMSMT:
    """Inverted index term -> sets, the exact answer RAMBO approximates."""

    def __init__(self, k: int):
        self.k = k
        self.post: dict[bytes, set[int]] = {}
        self.set_sizes: dict[int, int] = {}

    def add_seq(self, set_id: int, seq: bytes):
        for w in kmers_of(seq, self.k):
            self.post.setdefault(w, set()).add(set_id)

    def add_kmer_str(self, set_id: int, w: bytes):
        self.post.setdefault(canonical_str(w), set()).add(set_id)

    def query_kmer(self, w: bytes) -> set[int]:
        return set(self.post.get(canonical_str(w), ()))

    def query_seq(self, seq: bytes) -> set[int] | None:
        """Sets holding every k-mer of seq (Sec. 3.2.1); None if seq has none."""
        ks = kmers_of(seq, self.k)
        if not ks:
            return None
        ans = None
        for w in ks:
            s = self.post.get(w, set())
            ans = set(s) if ans is None else (ans & s)
            if not ans:
                return set()
        return ans

    def distinct_per_set(self, K: int) -> list[int]:
        n = [0] * K
        for sets in self.post.values():
            for i in sets:
                n[i] += 1
        return n

    def distinct_per_cell(self, phi_r, B: int) -> list[int]:
        """Distinct terms of the union of the sets in each cell of one
        repetition: n_b of the Bloom filter of cell b (Sec. 3)."""
        n = [0] * B
        for sets in self.post.values():
            for b in {int(phi_r[i]) for i in sets}:
                n[b] += 1
        return n
