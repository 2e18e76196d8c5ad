"""Python binding of librambo.so (include/rambo.h): argument marshalling only.

Device buffers are torch tensors on the GPU; every call passes their data
pointers and the current torch stream to the C ABI, and all work runs in the
library's HIP kernels.  There is no fallback: without the built library or a
GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librambo.so")

OK = 0
EINVAL = -22
ENOMEM = -12
ERANGE = -34
EIO = -5
EOVERFLOW = -75
EHIP = -1000
ECODE = -1001
ETIMEDOUT = -110
FLAG_IDENTITY_PARTITION = 1
FLAG_RAW_KEYS = 4   # terms are 64-bit keys (documents and word unigrams) passed as the k-mer codes
INSERT_AUTO, INSERT_DIRECT, INSERT_PARTITIONED, INSERT_PARTITIONED_WALKER = 0, 1, 2, 3
QUERY_AUTO, QUERY_WAVE_PER_READ, QUERY_QUEUE = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20   # RAMBO_NOALLOC_SCRATCH_BYTES
NO_KMER = -1   # UINT64_MAX viewed as int64

MAX_B = 4096
MAX_R = 16
MAX_RETA = 32


class RamboError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("K", ctypes.c_uint32), ("B", ctypes.c_uint32), ("R", ctypes.c_uint32),
                ("eta", ctypes.c_uint32), ("k", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("m", ctypes.c_uint64), ("seed", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("row_bits", ctypes.c_uint32), ("mask_words", ctypes.c_uint32),
                ("words_per_rep", ctypes.c_uint64), ("index_bytes", ctypes.c_uint64),
                ("index", ctypes.c_void_p)]


_lib = None

EXPORTS = {
    # name: (restype, argtypes)
    "rambo_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)]),
    "rambo_destroy": (None, [ctypes.c_void_p]),
    "rambo_insert_kmers": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "rambo_insert_seqs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "rambo_query_kmers": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "rambo_query_seqs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_query_termsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_extract_kmers": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                           ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_query_seqs_ids": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_query_seqs_ids_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                                    ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                    ctypes.c_void_p]),
    "rambo_query_seqs_ids_noalloc_max_reads": (ctypes.c_uint64, [ctypes.c_void_p]),
    "rambo_fill_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_query_kmers_plain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_query_seqs_plain": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_set_insert_policy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64]),
    "rambo_set_query_policy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]),
    "rambo_set_insert_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_get_insert_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "rambo_get_stage_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int]),
    "rambo_clear": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_fold": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p]),
    "rambo_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rambo_get_config": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "rambo_copy_index": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "rambo_get_partition": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_sync_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    # include/rambo_roofline.h
    "rambo_roofline_gather": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "rambo_roofline_atomic_or": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                ctypes.c_void_p]),
    "rambo_roofline_append": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.c_void_p]),
    "rambo_roofline_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    # include/rambo_serve.h
    "rambo_serve_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rambo_serve_destroy": (None, [ctypes.c_void_p]),
    "rambo_serve_submit": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "rambo_serve_submit_insert": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_uint64, ctypes.c_void_p]),
    "rambo_serve_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "rambo_serve_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int64]),
    "rambo_serve_inject_failures": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "rambo_serve_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint32)]),
    "rambo_serve_worker_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                ctypes.c_int]),
    "rambo_serve_batch_bytes": (ctypes.c_uint64, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]),
    "rambo_serve_mem_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_uint64)]),
}


class InsertTiles(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint32), ("stage_b_tile", ctypes.c_uint32), ("groups", ctypes.c_uint32),
                ("fine_bits", ctypes.c_uint32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_uint64), ("max_batch_bytes", ctypes.c_uint64),
                ("max_slots", ctypes.c_uint32), ("max_batch_reads", ctypes.c_uint32),
                ("use_graphs", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load librambo.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("librambo.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


_U32 = (torch.int32, torch.uint32)
_U64 = (torch.int64, torch.uint64)


def _dptr(t: torch.Tensor | None, dtypes, name: str) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


class Rambo:
    """A RAMBO index resident in GPU memory (one handle of the C ABI)."""

    def __init__(self, K: int, B: int, R: int, eta: int, k: int, m: int, seed: int, flags: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("Rambo needs a GPU")
        self.K, self.B, self.R, self.eta, self.k, self.m, self.seed = K, B, R, eta, k, m, seed
        cfg = Config(K, B, R, eta, k, flags, m, seed)
        h = ctypes.c_void_p()
        rc = lib().rambo_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise RamboError(rc, "rambo_create: " + (lib().rambo_last_error(None) or b"").decode())
        self._h = h
        self._refresh_info()

    @classmethod
    def load(cls, path: str) -> "Rambo":
        """An index resumed from a file written by save()."""
        if not torch.cuda.is_available():
            raise RuntimeError("Rambo needs a GPU")
        h = ctypes.c_void_p()
        rc = lib().rambo_load(str(path).encode(), ctypes.byref(h))
        if rc != OK:
            raise RamboError(rc, "rambo_load: " + (lib().rambo_last_error(None) or b"").decode())
        self = cls.__new__(cls)
        self._h = h
        cfg = Config()
        lib().rambo_get_config(h, ctypes.byref(cfg))
        self.K, self.B, self.R, self.eta, self.k, self.m, self.seed = (cfg.K, cfg.B, cfg.R, cfg.eta, cfg.k, cfg.m,
                                                                        cfg.seed)
        self._refresh_info()
        return self

    def save(self, path: str, stream=None):
        """Checkpoint the index to a file (waits for the work on stream)."""
        self._check(lib().rambo_save(self._h, str(path).encode(), _stream(stream)), "rambo_save")

    # lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().rambo_destroy(self._h)
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

    def _check(self, rc: int, what: str):
        if rc != OK:
            raise RamboError(rc, "%s: %s" % (what, (lib().rambo_last_error(self._h) or b"").decode()))

    # calls ------------------------------------------------------------------
    def insert_kmers(self, set_ids, offsets, codes, stream=None):
        n_sets = offsets.numel() - 1
        self._check(lib().rambo_insert_kmers(self._h, _dptr(set_ids, _U32, "set_ids"),
                                             _dptr(offsets, _U64, "offsets"), n_sets,
                                             _dptr(codes, _U64, "codes"), codes.numel(), _stream(stream)),
                    "rambo_insert_kmers")

    def insert_seqs(self, set_ids, offsets, chars, stream=None):
        n = offsets.numel() - 1
        self._check(lib().rambo_insert_seqs(self._h, _dptr(set_ids, _U32, "set_ids"),
                                            _dptr(offsets, _U64, "offsets"), n,
                                            _dptr(chars, (torch.uint8,), "chars"), chars.numel(),
                                            _stream(stream)),
                    "rambo_insert_seqs")

    def query_kmers(self, codes, out=None, stream=None, plain=False):
        n = codes.numel()
        if out is None:
            out = torch.empty((n, self.W), dtype=torch.int32, device=codes.device)
        fn = lib().rambo_query_kmers_plain if plain else lib().rambo_query_kmers
        self._check(fn(self._h, _dptr(codes, _U64, "codes"), n, _dptr(out, _U32, "out"), _stream(stream)),
                    "rambo_query_kmers")
        return out

    def query_termsets(self, offsets, codes, out=None, stream=None):
        """Sec. 3.2.1 for term sets: set q is codes[offsets[q]:offsets[q+1]];
        its answer holds the sets that hold every term (int64 device
        tensors in, [n_sets, W] int32 masks out)."""
        n = offsets.numel() - 1
        if out is None:
            out = torch.empty((n, self.W), dtype=torch.int32, device=offsets.device)
        self._check(lib().rambo_query_termsets(self._h, _dptr(offsets, _U64, "offsets"), n,
                                               _dptr(codes, _U64, "codes") if codes.numel() else None,
                                               codes.numel(), _dptr(out, _U32, "out"), _stream(stream)),
                    "rambo_query_termsets")
        return out

    def query_seqs(self, offsets, chars, out=None, nkmers=None, stream=None, plain=False, want_nkmers=True):
        n = offsets.numel() - 1
        dev = offsets.device
        if out is None:
            out = torch.empty((n, self.W), dtype=torch.int32, device=dev)
        if nkmers is None and want_nkmers:
            nkmers = torch.empty(n, dtype=torch.int32, device=dev)
        fn = lib().rambo_query_seqs_plain if plain else lib().rambo_query_seqs
        self._check(fn(self._h, _dptr(offsets, _U64, "offsets"), n, _dptr(chars, (torch.uint8,), "chars"),
                       chars.numel(), _dptr(out, _U32, "out"), _dptr(nkmers, _U32, "nkmers"), _stream(stream)),
                    "rambo_query_seqs")
        return out, nkmers

    def query_seqs_ids(self, offsets, chars, ids=None, nkmers=None, stream=None, id_offsets=None,
                       wait: bool = True):
        """Answers as ascending set-ID lists: (id_offsets int64 [n+1], ids
        int32 [total], window counts int32 [n]).  Synchronises `stream`; when
        the given (or first guessed) capacity is too small, calls again with
        exactly the capacity needed.  With wait=False: one asynchronous call
        into the given buffers (ids is the capacity), returned whole; the
        caller reads the list sizes from id_offsets and checks sync_status
        (EOVERFLOW: some list did not fit) once the stream is done."""
        n = offsets.numel() - 1
        id_off = id_offsets if id_offsets is not None else \
            torch.empty(max(n, 0) + 1, dtype=torch.int64, device=offsets.device)
        if id_off.numel() < n + 1:
            raise ValueError("id_offsets must hold n + 1 entries")
        if nkmers is None:
            nkmers = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
        if ids is None:
            ids = torch.empty(max(1024, 4 * n), dtype=torch.int32, device=offsets.device)
        if not wait:
            rc = lib().rambo_query_seqs_ids(self._h, _dptr(offsets, _U64, "offsets"), n,
                                            _dptr(chars, (torch.uint8,), "chars"), chars.numel(), id_off.data_ptr(),
                                            ids.data_ptr(), ids.numel(), _dptr(nkmers, _U32, "nkmers"),
                                            _stream(stream))
            self._check(rc, "rambo_query_seqs_ids")
            return id_off, ids, nkmers
        for _ in range(2):
            rc = lib().rambo_query_seqs_ids(self._h, _dptr(offsets, _U64, "offsets"), n,
                                            _dptr(chars, (torch.uint8,), "chars"), chars.numel(), id_off.data_ptr(),
                                            ids.data_ptr(), ids.numel(), _dptr(nkmers, _U32, "nkmers"),
                                            _stream(stream))
            self._check(rc, "rambo_query_seqs_ids")
            st = self.sync_status(stream)
            need = int(id_off[-1].item())
            if st == OK:
                return id_off, ids[:need], nkmers[:n]
            if st != EOVERFLOW:
                self._check(st, "rambo_query_seqs_ids")
            ids = torch.empty(need, dtype=torch.int32, device=offsets.device)
        raise RamboError(EOVERFLOW, "rambo_query_seqs_ids: capacity")

    def query_seqs_ids_noalloc(self, offsets, chars, id_offsets, ids, nkmers=None, stream=None):
        """rambo_query_seqs_ids into the caller's buffers, with the library's
        fixed per-GPU scratch instead of allocated state: id_offsets int64
        [n+1], ids int32 (its length is the capacity), nkmers int32 [n] or
        None.  Asynchronous on `stream`; an answer that did not fit shows as
        EOVERFLOW from sync_status."""
        n = offsets.numel() - 1
        if id_offsets.numel() < n + 1:
            raise ValueError("id_offsets must hold n + 1 entries")
        if nkmers is not None and nkmers.numel() < n:
            raise ValueError("nkmers must hold n entries")
        rc = lib().rambo_query_seqs_ids_noalloc(self._h, _dptr(offsets, _U64, "offsets"), n,
                                                _dptr(chars, (torch.uint8,), "chars"), chars.numel(),
                                                _dptr(id_offsets, _U64, "id_offsets"), _dptr(ids, _U32, "ids"),
                                                ids.numel(), _dptr(nkmers, _U32, "nkmers"), _stream(stream))
        self._check(rc, "rambo_query_seqs_ids_noalloc")

    def noalloc_max_reads(self) -> int:
        return int(lib().rambo_query_seqs_ids_noalloc_max_reads(self._h))

    def fill_counts(self, stream=None) -> torch.Tensor:
        """Set bits per cell, int64 [R, B] on the device."""
        out = torch.empty(self.R * self.B, dtype=torch.int64, device="cuda")
        self._check(lib().rambo_fill_counts(self._h, out.data_ptr(), _stream(stream)), "rambo_fill_counts")
        return out.view(self.R, self.B)

    def extract_kmers(self, offsets, chars, out=None, stream=None):
        n = chars.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.int64, device=chars.device)
        self._check(lib().rambo_extract_kmers(self._h, _dptr(offsets, _U64, "offsets"), offsets.numel() - 1,
                                              _dptr(chars, (torch.uint8,), "chars"), n,
                                              _dptr(out, _U64, "out"), _stream(stream)),
                    "rambo_extract_kmers")
        return out

    def set_insert_policy(self, mode: int = 0, scratch_bytes: int = 0):
        """INSERT_AUTO / INSERT_DIRECT / INSERT_PARTITIONED / INSERT_PARTITIONED_WALKER; same index bits."""
        self._check(lib().rambo_set_insert_policy(self._h, mode, scratch_bytes), "rambo_set_insert_policy")

    def set_insert_tiles(self, steps: int = 0, stage_b_tile: int = 0, groups: int = 0, fine_bits: int = 0):
        """Tile shapes of the partitioned insert (0 = automatic); same index bits."""
        t = InsertTiles(steps, stage_b_tile, groups, fine_bits)
        self._check(lib().rambo_set_insert_tiles(self._h, ctypes.byref(t)), "rambo_set_insert_tiles")

    def insert_tiles(self) -> dict:
        """The tile shapes the partitioned insert uses now."""
        t = InsertTiles()
        self._check(lib().rambo_get_insert_tiles(self._h, ctypes.byref(t)), "rambo_get_insert_tiles")
        return {f: getattr(t, f) for f, _ in InsertTiles._fields_}

    def set_query_policy(self, mode: int = 0, chunk_bytes: int = 0, waves_per_cu: int = 0):
        """QUERY_AUTO / QUERY_WAVE_PER_READ / QUERY_QUEUE; same answers."""
        self._check(lib().rambo_set_query_policy(self._h, mode, chunk_bytes, waves_per_cu),
                    "rambo_set_query_policy")

    def set_timing(self, enable: bool = True):
        self._check(lib().rambo_set_timing(self._h, int(enable)), "rambo_set_timing")

    def stage_times(self, max_stages: int = 32, calls: bool = False) -> dict:
        """Milliseconds per kernel name since the last call (HIP events);
        with calls, (milliseconds, launches) per name."""
        names = ctypes.create_string_buffer(48 * max_stages)
        ms = (ctypes.c_float * max_stages)()
        cnt = (ctypes.c_uint32 * max_stages)()
        n = lib().rambo_get_stage_times(self._h, names, ms, cnt, max_stages)
        if n < 0:
            self._check(n, "rambo_get_stage_times")
        raw = names.raw
        out = {}
        for i in range(min(n, max_stages)):
            name = raw[48 * i:48 * (i + 1)].split(b"\0")[0].decode()
            out[name] = (float(ms[i]), int(cnt[i])) if calls else float(ms[i])
        return out

    def _refresh_info(self):
        info = Info()
        lib().rambo_get_info(self._h, ctypes.byref(info))
        self.row_bits = info.row_bits
        self.W = info.mask_words
        self.words_per_rep = info.words_per_rep
        self.index_bytes = info.index_bytes
        self._index_ptr = info.index

    def fold(self, stream=None):
        """Folding over: B -> B/2 (synchronous)."""
        self._check(lib().rambo_fold(self._h, _stream(stream)), "rambo_fold")
        self.B //= 2
        self._refresh_info()

    def clear(self, stream=None):
        self._check(lib().rambo_clear(self._h, _stream(stream)), "rambo_clear")

    def sync_status(self, stream=None) -> int:
        """Synchronise and return (and clear) the sticky device error code."""
        return int(lib().rambo_sync_status(self._h, _stream(stream)))

    def partition(self):
        import numpy as np
        out = np.zeros(self.R * self.K, dtype=np.uint32)
        self._check(lib().rambo_get_partition(self._h, out.ctypes.data), "rambo_get_partition")
        return out.reshape(self.R, self.K)

    def index_words(self, word_offset: int = 0, n_words: int | None = None, stream=None) -> torch.Tensor:
        """A device copy of index words [word_offset, word_offset + n_words)
        as int32 (all R * words_per_rep words by default)."""
        total = self.index_bytes // 4
        if n_words is None:
            n_words = total - word_offset
        out = torch.empty(n_words, dtype=torch.int32, device="cuda")
        self._check(lib().rambo_copy_index(self._h, word_offset, n_words, out.data_ptr(), _stream(stream)),
                    "rambo_copy_index")
        return out


class Server:
    """A continuous-batching query server on a resident index
    (include/rambo_serve.h).  Requests are host numpy arrays; the index
    handle must not be used for anything else until close()."""

    def __init__(self, index: Rambo, mem_budget: int = 0, max_batch_bytes: int = 0, max_slots: int = 0,
                 max_batch_reads: int = 0, use_graphs: bool = False):
        self.index = index
        cfg = ServeConfig(mem_budget, max_batch_bytes, max_slots, max_batch_reads, int(use_graphs), 0)
        h = ctypes.c_void_p()
        index._check(lib().rambo_serve_create(index._h, ctypes.byref(cfg), ctypes.byref(h)), "rambo_serve_create")
        self._s = h

    def close(self):
        if getattr(self, "_s", None):
            lib().rambo_serve_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, offsets, chars) -> int:
        """Queue reads chars[offsets[i]:offsets[i+1]] (host uint64 offsets,
        uint8 bytes); returns the request id."""
        import numpy as np
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        ch = np.ascontiguousarray(np.frombuffer(chars, np.uint8) if isinstance(chars, (bytes, bytearray)) else chars,
                                  dtype=np.uint8)
        n = len(off) - 1
        rid = lib().rambo_serve_submit(self._s, off.ctypes.data, n, ch.ctypes.data if ch.size else None)
        if rid < 0:
            raise RamboError(int(rid), "rambo_serve_submit")
        return int(rid)

    def submit_insert(self, set_ids, offsets, chars) -> int:
        """Queue the insertion of sequences chars[offsets[s]:offsets[s+1]]
        into sets set_ids[s] (host arrays); it takes effect between the
        requests submitted before and after it.  Returns the request id (for
        wait_insert)."""
        import numpy as np
        ids = np.ascontiguousarray(set_ids, dtype=np.uint32)
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        ch = np.ascontiguousarray(chars, dtype=np.uint8)
        rid = lib().rambo_serve_submit_insert(self._s, ids.ctypes.data, off.ctypes.data, ids.size,
                                              ch.ctypes.data if ch.size else None)
        if rid < 0:
            raise RamboError(int(rid), "rambo_serve_submit_insert")
        return int(rid)

    def wait_insert(self, rid: int, timeout_us: int = -1) -> float:
        """Wait for insert request rid; raises on its error status.  Returns
        its latency in ms."""
        lat = ctypes.c_double()
        rc = lib().rambo_serve_wait(self._s, rid, None, None, ctypes.byref(lat), timeout_us)
        if rc != OK:
            raise RamboError(rc, "rambo_serve_wait (insert)")
        return lat.value

    def wait(self, rid: int, n_reads: int, timeout_us: int = -1):
        """(masks [n_reads, W] uint32, window counts [n_reads] uint32,
        latency in ms) of request rid."""
        import numpy as np
        masks = np.zeros((n_reads, self.index.W), dtype=np.uint32)
        nk = np.zeros(n_reads, dtype=np.uint32)
        lat = ctypes.c_double()
        rc = lib().rambo_serve_wait(self._s, rid, masks.ctypes.data, nk.ctypes.data, ctypes.byref(lat), timeout_us)
        if rc != OK:
            raise RamboError(rc, "rambo_serve_wait")
        return masks, nk, lat.value

    def replay(self, req_reads, read_offsets, chars, arrival_s, with_queue=False):
        """Native open-loop drive (rambo_serve_replay): request i = reads
        req_reads[i] .. req_reads[i+1]-1 of the host CSR (read_offsets,
        chars), submitted at arrival_s[i] seconds.  Returns (latencies in ms,
        answer checksum), and with with_queue the host-queue part of each
        latency (ms) as a third item."""
        import numpy as np
        rr = np.ascontiguousarray(req_reads, dtype=np.uint64)
        off = np.ascontiguousarray(read_offsets, dtype=np.uint64)
        ch = np.ascontiguousarray(chars, dtype=np.uint8)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        n = rr.size - 1
        lat = np.zeros(n, dtype=np.float64)
        qms = np.zeros(n, dtype=np.float64)
        ck = ctypes.c_uint64()
        rc = lib().rambo_serve_replay(self._s, n, rr.ctypes.data, off.ctypes.data, ch.ctypes.data, arr.ctypes.data,
                                      lat.ctypes.data, qms.ctypes.data, ctypes.byref(ck))
        if rc != OK:
            raise RamboError(rc, "rambo_serve_replay")
        return (lat, ck.value, qms) if with_queue else (lat, ck.value)

    def worker_stats(self, reset: bool = False) -> dict:
        """Worker-thread maxima in microseconds: loop gap, batch enqueue,
        completion query (rambo_serve_worker_stats)."""
        g, e, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().rambo_serve_worker_stats(self._s, ctypes.byref(g), ctypes.byref(e), ctypes.byref(q), int(reset))
        if rc != OK:
            raise RamboError(rc, "rambo_serve_worker_stats")
        return {"max_loop_gap_us": g.value, "max_enqueue_us": e.value, "max_query_us": q.value}

    def inject_failures(self, n_batches: int):
        """Test hook: the next n_batches batches fail before launch (their
        requests are answered with RAMBO_EHIP)."""
        rc = lib().rambo_serve_inject_failures(self._s, n_batches)
        if rc != OK:
            raise RamboError(rc, "rambo_serve_inject_failures")

    def stats(self) -> dict:
        b, q, r = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        sl = ctypes.c_uint32()
        lib().rambo_serve_stats(self._s, ctypes.byref(b), ctypes.byref(q), ctypes.byref(r), ctypes.byref(sl))
        bud, use, pk, wt = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        lib().rambo_serve_mem_stats(self._s, ctypes.byref(bud), ctypes.byref(use), ctypes.byref(pk), ctypes.byref(wt))
        return {"batches": b.value, "requests": q.value, "reads": r.value, "slots": sl.value,
                "mem_budget": bud.value, "mem_in_use": use.value, "mem_peak": pk.value, "mem_waits": wt.value}
