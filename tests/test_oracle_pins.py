"""Pins of the oracle's building blocks against values fixed outside it.

* splitmix64 / mix64: the generator's published known-answer vector.
* k-mer codes: hand-worked strings, Python's base-4 integer parser, and
  string-level reverse complements (oracle.bruteforce).
* partition hash: hand-worked closed forms of (a i + b) mod (2^61 - 1) mod B,
  the partition invariant and the 1/B collision rate of a 2-universal family
  (Sec. 3.1; Sec. 5.2 and the appendix state the 1/B collision probability).
* Bloom-filter positions: range, the power-of-two special case, a
  chi-square uniformity test, and the pairwise collision bound of the
  multiply-shift family (at most 2/m over random odd multipliers,
  Dietzfelbinger et al. 1997).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_splitmix64_known_answer():
    rows = _rows("splitmix64_kat.txt")
    seed = int(rows[0][1])
    want = [int(r[0]) for r in rows[1:]]
    assert oracle.splitmix64_stream(seed, len(want)) == want
    # the generator's output is mix64 of the advanced state
    assert oracle.mix64((seed + 0x9E3779B97F4A7C15) % (1 << 64)) == want[0]


def test_mix64_avalanche():
    rng = np.random.default_rng(5)
    flips = []
    for x in rng.integers(0, 1 << 63, size=200, dtype=np.uint64):
        x = int(x)
        hx = oracle.mix64(x)
        for bit in (0, 7, 31, 40, 63):
            flips.append(bin(hx ^ oracle.mix64(x ^ (1 << bit))).count("1"))
    assert 30 < np.mean(flips) < 34


def test_kmer_codes_hand_worked():
    for s, code, rc, can in _rows("kmer_codes.txt"):
        k = len(s)
        assert oracle.encode_kmer(s) == int(code), s
        assert oracle.revcomp(int(code), k) == int(rc), s
        assert oracle.canonical(int(code), k) == int(can), s


def test_kmer_codes_match_base4_parser():
    rng = np.random.default_rng(11)
    for k in (1, 2, 5, 15, 16, 21, 31, 32):
        for _ in range(200):
            w = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=k).tobytes()
            code = oracle.encode_kmer(w)
            assert code == bf.code_of_str(w)
            assert oracle.revcomp(code, k) == bf.code_of_str(bf.revcomp_str(w))
            assert oracle.canonical(code, k) == bf.code_of_str(bf.canonical_str(w))
            assert oracle.revcomp(oracle.revcomp(code, k), k) == code


def test_invalid_bytes_break_window():
    for s in (b"ACGN", b"NACG", b"AC-T", b"ACGU"):
        assert oracle.encode_kmer(s) is None


def test_extract_matches_string_windows():
    rng = np.random.default_rng(3)
    k = 7
    seqs = []
    for L in (0, 3, 6, 7, 8, 30, 64, 100):
        s = bytearray(rng.choice(np.frombuffer(b"ACGTacgt", np.uint8), size=L).tobytes())
        for p in rng.integers(0, max(L, 1), size=L // 20):
            s[p] = ord("N")
        seqs.append(bytes(s))
    offsets = np.zeros(len(seqs) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(s) for s in seqs])
    chars = np.frombuffer(b"".join(seqs), np.uint8)
    out = oracle.extract(offsets, chars, k)
    for si, s in enumerate(seqs):
        base = int(offsets[si])
        for t in range(len(s)):
            w = s[t:t + k]
            if len(w) == k and all(c in b"ACGTacgt" for c in w):
                assert int(out[base + t]) == bf.code_of_str(bf.canonical_str(w))
            else:
                assert out[base + t] == oracle.NO_KMER


def test_partition_closed_forms():
    for a, b, i, B, e in _rows("partition_modp.txt"):
        assert oracle.partition_value(int(a), int(b), int(i), int(B)) == int(e)


def test_partition_invariant_and_seed_determinism():
    K, B, R = 300, 17, 5
    idx1 = oracle.OracleIndex(K, B, R, 2, 31, 1024, seed=42)
    idx2 = oracle.OracleIndex(K, B, R, 2, 31, 1024, seed=42)
    idx3 = oracle.OracleIndex(K, B, R, 2, 31, 1024, seed=43)
    a1, b1, s1, phi1 = idx1.params()
    a2, b2, s2, phi2 = idx2.params()
    assert (phi1 == phi2).all() and (s1 == s2).all() and (a1 == a2).all()
    assert not (phi1 == idx3.phi()).all()
    assert phi1.shape == (R, K) and phi1.max() < B
    P = (1 << 61) - 1
    assert all(1 <= int(a) < P for a in a1) and all(0 <= int(b) < P for b in b1)
    # seeds come from one splitmix64 stream in the documented order
    stream = oracle.splitmix64_stream(42, 2 * R + R * 2)
    for r in range(R):
        assert int(a1[r]) == 1 + stream[2 * r] % (P - 1)
        assert int(b1[r]) == stream[2 * r + 1] % P
    assert [int(v) for v in s1.reshape(-1)] == stream[2 * R:]
    # phi_r(i) is the partition value of the stream parameters
    for r in range(R):
        for i in (0, 1, 77, K - 1):
            assert phi1[r, i] == oracle.partition_value(int(a1[r]), int(b1[r]), i, B)


def test_partition_collision_rate_is_one_over_B():
    B = 10
    n_seeds = 3000
    coll = 0
    for sd in range(n_seeds):
        phi = oracle.OracleIndex(1001, B, 1, 1, 31, 64, seed=10_000 + sd).phi()
        coll += int(phi[0, 3] == phi[0, 1000])
    p = coll / n_seeds
    sd = np.sqrt(0.1 * 0.9 / n_seeds)
    assert abs(p - 1 / B) < 4 * sd


def test_identity_partition_flag():
    idx = oracle.OracleIndex(20, 20, 2, 1, 31, 64, seed=1, flags=oracle.FLAG_IDENTITY_PARTITION)
    phi = idx.phi()
    assert (phi == np.arange(20)[None, :]).all()


def test_position_range_and_power_of_two_case():
    rng = np.random.default_rng(9)
    for x in rng.integers(0, 1 << 62, size=200, dtype=np.uint64):
        x = int(x)
        for s in (0, 12345, (1 << 64) - 1):
            v = ((s | 1) * oracle.mix64(x)) % (1 << 64)
            for t in (6, 18, 28, 40):
                assert oracle.position(x, s, 1 << t) == v >> (64 - t)
            for m in (64, 1000, 3 * (1 << 20) + 7):
                assert 0 <= oracle.position(x, s, m) < m


def test_position_uniformity_chi2():
    from scipy import stats
    m = 1 << 10
    n = 200_000
    # consecutive codes are the hardest input for a weak mixer
    counts = np.zeros(m, np.int64)
    for x in range(n):
        counts[oracle.position(x, 0x1234ABCD, m)] += 1
    chi2 = ((counts - n / m) ** 2 / (n / m)).sum()
    assert stats.chi2.sf(chi2, m - 1) > 1e-4


def test_position_pair_collision_rate():
    # multiply-shift is 2-universal up to a factor 2: for fixed distinct keys
    # and a random odd multiplier, P[pos(x) = pos(y)] <= 2/m; averaged over
    # key pairs it is close to 1/m.  Codes one apart are the hardest pairs.
    m = 1 << 8
    rng = np.random.default_rng(11)
    seeds = [int(v) for v in rng.integers(0, 1 << 63, size=4000, dtype=np.uint64)]
    total, hits = 0, 0
    for x in [0, 1, 12345, (1 << 61) + 3, 4 ** 31 - 2]:
        for y in (x + 1, x + 2, x ^ (1 << 40)):
            c = sum(oracle.position(x, s, m) == oracle.position(y, s, m) for s in seeds)
            assert c / len(seeds) <= 2.0 / m + 4 * np.sqrt(2.0 / m / len(seeds))
            hits += c
            total += len(seeds)
    p = hits / total
    assert abs(p - 1.0 / m) <= 4 * np.sqrt(1.0 / m / total) + 0.25 / m


def test_mask_bit_order_and_padding():
    K = 70
    m = oracle.ids_to_mask([0, 31, 32, 69], K)
    assert m.tolist() == [1 | (1 << 31), 1, 1 << 5]
    assert oracle.mask_to_ids(m, K) == [0, 31, 32, 69]


def test_create_rejects_bad_config():
    bad = [dict(K=0), dict(B=0), dict(B=11), dict(R=0), dict(eta=0), dict(k=0), dict(k=33), dict(m=63)]
    for b in bad:
        cfg = dict(K=10, B=5, R=2, eta=2, k=31, m=1024)
        cfg.update(b)
        with pytest.raises(ValueError):
            oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed=0)
