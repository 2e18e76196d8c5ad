"""RAMBO oracle: plain CPU reference for the GPU library (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never calls it.

``rambo_oracle.c`` holds the index itself (separate Bloom filter per cell,
Sec. 3 / Alg. 1 / Alg. 2 of arXiv 1910.02611); this module is its ctypes
binding.  ``bruteforce`` holds the exact multiple-set-membership answer
(Sec. 1, MSMT statement) and ``fpr`` the false-positive predictions of
Sec. 2 and Lemma 4.1.  None of them share code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rambo_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAG_IDENTITY_PARTITION = 1
FLAG_NO_FILTERS = 2   # parameters only, for the row scans of indexes larger than host memory
FLAG_RAW_KEYS = 4     # terms are arbitrary 64-bit keys (documents and word unigrams), not k-mer codes
NO_KMER = np.uint64(0xFFFFFFFFFFFFFFFF)

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        vp = ctypes.c_void_p
        sig = {
            "orc_mix64": (u64, [u64]),
            "orc_splitmix64_next": (u64, [_u64p]),
            "orc_partition_value": (u32, [u64, u64, u64, u32]),
            "orc_position": (u64, [u64, u64, u64]),
            "orc_encode_kmer": (i32, [ctypes.c_char_p, u32, _u64p]),
            "orc_revcomp": (u64, [u64, u32]),
            "orc_canonical": (u64, [u64, u32]),
            "orc_extract": (None, [vp, vp, u64, u32, vp]),
            "orc_create": (i32, [u32, u32, u32, u32, u32, u64, u64, u32, ctypes.POINTER(vp)]),
            "orc_destroy": (None, [vp]),
            "orc_params": (None, [vp, vp, vp, vp, vp]),
            "orc_insert_kmer": (i32, [vp, u32, u64]),
            "orc_insert_seq": (i32, [vp, u32, vp, u64]),
            "orc_insert_seqs": (i32, [vp, vp, vp, vp, u64, i32]),
            "orc_insert_kmers": (i32, [vp, vp, vp, vp, u64, i32]),
            "orc_query_cells": (None, [vp, u64, vp]),
            "orc_query_kmer": (i32, [vp, u64, vp]),
            "orc_query_kmers": (None, [vp, vp, u64, vp, i32]),
            "orc_query_seq": (u64, [vp, vp, u64, vp]),
            "orc_query_seqs": (i32, [vp, vp, vp, u64, vp, vp, i32]),
            "orc_fill_counts": (None, [vp, vp]),
            "orc_copy_bfu": (None, [vp, u32, u32, vp]),
            "orc_bits_at": (None, [vp, u32, vp, u64, vp]),
            "orc_max_threads": (i32, []),
            "orc_fold": (i32, [vp]),
            "orc_set_partition": (i32, [vp, vp]),
            "orc_scan_rows": (i32, [vp, vp, vp, vp, u64, u64, vp, vp, u64, vp, i32, i32]),
            "orc_window_keys": (u64, [vp, vp, vp, u64, vp, u64]),
            "orc_cell_bits": (i32, [vp, u32, u32, vp, vp, vp, u64, vp, i32]),
            "orc_query_seqs_rows": (i32, [vp, vp, vp, u64, vp, u64, vp, vp, vp, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ------------------------------------------------------------------ scalars

def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def splitmix64_stream(seed: int, n: int) -> list[int]:
    st = ctypes.c_uint64(seed)
    return [int(lib().orc_splitmix64_next(ctypes.byref(st))) for _ in range(n)]


def partition_value(a: int, b: int, i: int, B: int) -> int:
    return int(lib().orc_partition_value(a, b, i, B))


def position(x: int, seed: int, m: int) -> int:
    return int(lib().orc_position(x, seed, m))


def encode_kmer(s: bytes, k: int | None = None):
    """Code of the first k bytes of s, or None if one of them is not a base."""
    if isinstance(s, str):
        s = s.encode()
    k = len(s) if k is None else k
    out = ctypes.c_uint64(0)
    ok = lib().orc_encode_kmer(s, k, ctypes.byref(out))
    return int(out.value) if ok else None


def revcomp(code: int, k: int) -> int:
    return int(lib().orc_revcomp(code, k))


def canonical(code: int, k: int) -> int:
    return int(lib().orc_canonical(code, k))


def extract(offsets: np.ndarray, chars: np.ndarray, k: int) -> np.ndarray:
    """Canonical code of the window starting at every base, NO_KMER where none."""
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    out = np.empty(chars.size, dtype=np.uint64)
    lib().orc_extract(_ptr(offsets), _ptr(chars), offsets.size - 1, k, _ptr(out))
    return out


# ------------------------------------------------------------------- index

class OracleIndex:
    """R x B separate Bloom filters of m bits each (Sec. 3)."""

    def __init__(self, K, B, R, eta, k, m, seed, flags=0):
        self.K, self.B, self.R, self.eta, self.k, self.m = K, B, R, eta, k, m
        self.seed, self.flags = seed, flags
        self.W = (K + 31) // 32
        h = ctypes.c_void_p()
        rc = lib().orc_create(K, B, R, eta, k, m, seed, flags, ctypes.byref(h))
        if rc != 0:
            raise ValueError("orc_create failed (%d)" % rc)
        self._h = h

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # parameters
    def params(self):
        a = np.zeros(self.R, np.uint64)
        b = np.zeros(self.R, np.uint64)
        s = np.zeros(self.R * self.eta, np.uint64)
        phi = np.zeros(self.R * self.K, np.uint32)
        lib().orc_params(self._h, _ptr(a), _ptr(b), _ptr(s), _ptr(phi))
        return a, b, s.reshape(self.R, self.eta), phi.reshape(self.R, self.K)

    def phi(self) -> np.ndarray:
        return self.params()[3]

    # insertion (Alg. 1)
    def insert_kmer(self, set_id: int, code: int) -> int:
        return int(lib().orc_insert_kmer(self._h, set_id, code))

    def insert_seq(self, set_id: int, seq: bytes) -> int:
        buf = np.frombuffer(seq, dtype=np.uint8).copy()
        return int(lib().orc_insert_seq(self._h, set_id, _ptr(buf), buf.size))

    def insert_seqs(self, set_ids, offsets, chars, nthreads=0) -> int:
        set_ids = np.ascontiguousarray(set_ids, np.uint32)
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        assert offsets.size == set_ids.size + 1 and int(offsets[-1]) <= chars.size
        return int(lib().orc_insert_seqs(self._h, _ptr(set_ids), _ptr(offsets), _ptr(chars),
                                         set_ids.size, nthreads))

    def insert_kmers(self, set_ids, offsets, codes, nthreads=0) -> int:
        set_ids = np.ascontiguousarray(set_ids, np.uint32)
        offsets = np.ascontiguousarray(offsets, np.uint64)
        codes = np.ascontiguousarray(codes, np.uint64)
        assert offsets.size == set_ids.size + 1 and int(offsets[-1]) <= codes.size
        return int(lib().orc_insert_kmers(self._h, _ptr(set_ids), _ptr(offsets), _ptr(codes),
                                          set_ids.size, nthreads))

    # query (Alg. 2, Sec. 3.2.1)
    def query_cells(self, code: int) -> np.ndarray:
        G = np.zeros(self.R * self.B, np.uint8)
        lib().orc_query_cells(self._h, code, _ptr(G))
        return G.reshape(self.R, self.B)

    def query_kmer(self, code: int) -> np.ndarray:
        out = np.zeros(self.W, np.uint32)
        lib().orc_query_kmer(self._h, code, _ptr(out))
        return out

    def query_kmers(self, codes, nthreads=0) -> np.ndarray:
        codes = np.ascontiguousarray(codes, np.uint64)
        out = np.zeros((codes.size, self.W), np.uint32)
        lib().orc_query_kmers(self._h, _ptr(codes), codes.size, _ptr(out), nthreads)
        return out

    def query_seq(self, seq: bytes):
        buf = np.frombuffer(seq, dtype=np.uint8).copy()
        out = np.zeros(self.W, np.uint32)
        n = lib().orc_query_seq(self._h, _ptr(buf), buf.size, _ptr(out))
        return out, int(n)

    def query_seqs(self, offsets, chars, nthreads=0):
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        n = offsets.size - 1
        out = np.zeros((n, self.W), np.uint32)
        nk = np.zeros(n, np.uint64)
        rc = lib().orc_query_seqs(self._h, _ptr(offsets), _ptr(chars), n, _ptr(out), _ptr(nk), nthreads)
        if rc != 0:
            raise ValueError("orc_query_seqs failed (%d)" % rc)
        return out, nk

    # inspection
    def fill_counts(self) -> np.ndarray:
        out = np.zeros(self.R * self.B, np.uint64)
        lib().orc_fill_counts(self._h, _ptr(out))
        return out.reshape(self.R, self.B)

    def bfu_words(self, r: int, b: int) -> np.ndarray:
        out = np.zeros((self.m + 63) // 64, np.uint64)
        lib().orc_copy_bfu(self._h, r, b, _ptr(out))
        return out

    def bfu_bits(self, r: int, b: int) -> np.ndarray:
        """The m bits of cell (r, b) as a uint8 0/1 vector."""
        w = self.bfu_words(r, b)
        return np.unpackbits(w.view(np.uint8), bitorder="little")[: self.m]

    def bits_at(self, r: int, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, np.uint64)
        out = np.zeros((rows.size, self.B), np.uint8)
        lib().orc_bits_at(self._h, r, _ptr(rows), rows.size, _ptr(out))
        return out

    def fold(self):
        """Folding over: B -> B/2 (cell b + B/2 OR-ed into cell b)."""
        rc = lib().orc_fold(self._h)
        if rc != 0:
            raise ValueError("orc_fold failed (%d)" % rc)
        self.B //= 2

    def set_partition(self, phi):
        """Install the partition phi[r, i] (an empty index only; test hook)."""
        phi = np.ascontiguousarray(phi, np.uint32)
        rc = lib().orc_set_partition(self._h, _ptr(phi))
        if rc != 0:
            raise ValueError("orc_set_partition failed (%d)" % rc)

    # rows of indexes too large for host memory (works with FLAG_NO_FILTERS)
    @property
    def row_words(self) -> int:
        return (self.B + 63) // 64

    def window_keys(self, offsets, chars) -> np.ndarray:
        """Row keys r*m + pos_{r,j}(x) of every valid window of every read."""
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        n = offsets.size - 1
        cnt = int(lib().orc_window_keys(self._h, _ptr(offsets), _ptr(chars), n, None, 0))
        out = np.zeros(max(cnt, 1), np.uint64)
        lib().orc_window_keys(self._h, _ptr(offsets), _ptr(chars), n, _ptr(out), cnt)
        return out[:cnt]

    def scan_rows(self, set_ids, offsets, chars, D: int = 0, keys=None, nthreads=0, progress=False):
        """One pass over the inserted sets: (rows p % D == 0 of every
        repetition as [R, m/D, BW] uint64 or None, rows of the given
        ascending distinct keys as [n_keys, BW] uint64 or None)."""
        set_ids = np.ascontiguousarray(set_ids, np.uint32)
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        BW = self.row_words
        sampled = np.zeros((self.R, self.m // D, BW), np.uint64) if D else None
        keys = None if keys is None else np.ascontiguousarray(keys, np.uint64)
        rows = np.zeros((keys.size, BW), np.uint64) if keys is not None else None
        rc = lib().orc_scan_rows(self._h, _ptr(set_ids), _ptr(offsets), _ptr(chars), set_ids.size, D,
                                 _ptr(sampled) if sampled is not None else None,
                                 _ptr(keys) if keys is not None else None, 0 if keys is None else keys.size,
                                 _ptr(rows) if rows is not None else None, nthreads, int(progress))
        if rc != 0:
            raise ValueError("orc_scan_rows failed (%d)" % rc)
        return sampled, rows

    def cell_bits(self, r: int, b: int, set_ids, offsets, chars, nthreads=0) -> np.ndarray:
        """The BFU of cell (r, b) built from the given sequences (Alg. 1 for
        that one cell): ceil(m/64) uint64 words, bit p of word p/64."""
        set_ids = np.ascontiguousarray(set_ids, np.uint32)
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        out = np.zeros((self.m + 63) // 64, np.uint64)
        rc = lib().orc_cell_bits(self._h, r, b, _ptr(set_ids), _ptr(offsets), _ptr(chars), set_ids.size,
                                 _ptr(out), nthreads)
        if rc != 0:
            raise ValueError("orc_cell_bits failed (%d)" % rc)
        return out

    def members_from_cells(self, offsets, chars, cells) -> np.ndarray:
        """Whether one set s is in the Sec. 3.2.1 answer of each read, from
        the R cells that hold it (cells[r]: the BFU words of cell
        (r, phi_r(s))).  Alg. 2 answers the intersection over r of the union
        of the sets of the passing cells; s lies in exactly one cell per
        repetition, so it is in the answer of a term iff every one of its R
        cells passes (all eta bits set), and in a read's answer iff that holds
        for every valid window.  A read with no valid window answers the
        empty set."""
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        n = offsets.size - 1
        out = np.zeros(n, bool)
        base = (np.arange(self.R, dtype=np.uint64) * np.uint64(self.m))[None, :, None]
        for i in range(n):
            o = np.array([0, offsets[i + 1] - offsets[i]], np.uint64)
            keys = self.window_keys(o, chars[int(offsets[i]):int(offsets[i + 1])])
            if keys.size == 0:
                continue
            pos = keys.reshape(-1, self.R, self.eta) - base
            ok = True
            for r in range(self.R):
                p = pos[:, r, :].ravel()
                ok = ok and bool(((cells[r][p // np.uint64(64)] >> (p % np.uint64(64))) & np.uint64(1)).all())
            out[i] = ok
        return out

    def query_seqs_rows(self, offsets, chars, keys, rows, nthreads=0):
        """Sec. 3.2.1 answers of reads with the filter bits read from rows
        (as scan_rows returns them): (masks [n, W], window counts [n])."""
        offsets = np.ascontiguousarray(offsets, np.uint64)
        chars = np.ascontiguousarray(chars, np.uint8)
        keys = np.ascontiguousarray(keys, np.uint64)
        rows = np.ascontiguousarray(rows, np.uint64)
        n = offsets.size - 1
        out = np.zeros((n, self.W), np.uint32)
        nk = np.zeros(n, np.uint64)
        rc = lib().orc_query_seqs_rows(self._h, _ptr(offsets), _ptr(chars), n, _ptr(keys), keys.size, _ptr(rows),
                                       _ptr(out), _ptr(nk), nthreads)
        if rc != 0:
            raise ValueError("orc_query_seqs_rows failed (%d): a needed row is missing" % rc)
        return out, nk


def max_threads() -> int:
    return int(lib().orc_max_threads())


def mask_to_ids(mask_row: np.ndarray, K: int) -> list[int]:
    """Set IDs of one K-bit mask (bit i of word i/32, LSB first)."""
    bits = np.unpackbits(np.ascontiguousarray(mask_row, np.uint32).view(np.uint8), bitorder="little")
    return [int(i) for i in np.nonzero(bits[:K])[0]]


def ids_to_mask(ids, K: int) -> np.ndarray:
    W = (K + 31) // 32
    bits = np.zeros(W * 32, np.uint8)
    for i in ids:
        bits[i] = 1
    return np.packbits(bits, bitorder="little").view(np.uint32).copy()
