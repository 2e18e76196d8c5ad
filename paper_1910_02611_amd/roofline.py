"""Measured memory ceilings for the RAMBO access patterns (rambo_roofline.h).

measure(buf_bytes) runs, over one device buffer of buf_bytes:
  * random aligned gathers of 4..256 bytes (the probe of a row, Alg. 2),
  * random non-returning 32-bit atomicOr (the insertion of a bit, Alg. 1),
  * a streaming copy (sequential reference),
and returns accesses per second and bytes per second for each.
append(buf_bytes, streams) measures the binning's write pattern: runs of 16
words appended to `streams` per-workgroup chunks, with runs starting inside
64-byte segments (as at a running cursor) and aligned to them.
"""
from __future__ import annotations

import sys

import torch

from .rambo import lib

GATHER_SIZES = (4, 8, 16, 32, 64, 128, 256)


def _time(fn, reps=3):
    stream = torch.cuda.current_stream()
    fn()  # warm
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        s.record(stream)
        fn()
        e.record(stream)
        e.synchronize()
        best = min(best, s.elapsed_time(e) / 1e3)
    return best


def measure(buf_bytes: int, n_access: int = 1 << 27, sizes=GATHER_SIZES, buf: torch.Tensor | None = None):
    L = lib()
    st = torch.cuda.current_stream().cuda_stream
    if buf is None:
        buf = torch.empty(buf_bytes // 4, dtype=torch.int32, device="cuda")
        buf.zero_()
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    nbytes = buf.numel() * 4
    out = {"buffer_bytes": nbytes, "n_access": n_access, "gather": {}}
    for G in sizes:
        def f(G=G):
            rc = L.rambo_roofline_gather(buf.data_ptr(), nbytes - nbytes % G, G, n_access, 12345 + G,
                                         sink.data_ptr(), st)
            assert rc == 0
        t = _time(f)
        out["gather"][str(G)] = {"accesses_per_s": n_access / t, "useful_GBps": n_access * G / t / 1e9,
                                 "sector64_GBps": n_access * max(G, 64) / t / 1e9}

    def a():
        assert L.rambo_roofline_atomic_or(buf.data_ptr(), buf.numel(), n_access, 777, st) == 0
    t = _time(a)
    out["atomic_or"] = {"accesses_per_s": n_access / t, "rmw_sector64_GBps": n_access * 128 / t / 1e9}

    half = (nbytes // 2) // 16 * 16

    def c():
        assert L.rambo_roofline_copy(buf.data_ptr(), buf.data_ptr() + half, half, st) == 0
    t = _time(c)
    out["copy"] = {"bytes": half, "GBps_read_plus_write": 2 * half / t / 1e9}
    return out


def append(buf_bytes: int, streams: int, run: int = 16, n_workgroups: int = 256,
           buf: torch.Tensor | None = None) -> dict:
    """Bytes per second of the binning's write pattern (rambo_roofline_append)
    over one buffer: misaligned (runs start 0..15 words into a segment) and
    aligned runs."""
    import ctypes
    L = lib()
    st = torch.cuda.current_stream().cuda_stream
    if buf is None:
        buf = torch.empty(buf_bytes // 4, dtype=torch.int32, device="cuda")
    out = {"buffer_bytes": buf.numel() * 4, "streams": streams, "run_words": run, "workgroups": n_workgroups}
    for name, mis in (("misaligned", 1), ("aligned", 0)):
        words = ctypes.c_uint64(0)

        def f(mis=mis, words=words):
            rc = L.rambo_roofline_append(buf.data_ptr(), buf.numel(), streams, run, mis, n_workgroups,
                                         ctypes.byref(words), st)
            assert rc == 0
        t = _time(f)
        out[name] = {"bytes": words.value * 4, "GBps": words.value * 4 / t / 1e9}
    return out


if __name__ == "__main__":
    import json
    gib = float(sys.argv[1]) if len(sys.argv) > 1 else 8.0
    print(json.dumps(measure(int(gib * 2**30))))
