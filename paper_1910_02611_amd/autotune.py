"""Tile autotuner for the batched query launches.

Sweeps the work-queue shape of rambo_query_seqs (bytes per work item,
persistent waves per compute unit) on a representative batch, times every
candidate with HIP events on the current stream, keeps the fastest, and
caches the choice in a JSON file keyed by device and index shape, so a later
run (or the serving loop) starts from it.  Every candidate computes the same
answers; the sweep checks that too.
"""
from __future__ import annotations

import json
import os

import torch

from . import rambo as rb

CHUNKS = (256, 512, 1024, 2048, 4096)
WAVES_PER_CU = (8, 16, 32)


def cache_path() -> str:
    return os.environ.get("RAMBO_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rambo_tune.json"))


def _key(g: rb.Rambo, tag: str) -> str:
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s|%s|K%d-B%d-R%d-e%d-m%d|%s" % (dev.name, getattr(dev, "gcnArchName", ""), g.K, g.B, g.R, g.eta,
                                             g.m, tag)


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_query_seqs(g: rb.Rambo, offsets, chars, out, nk, reps: int = 3) -> float:
    """Best of reps, in seconds, of one batched rambo_query_seqs call."""
    stream = torch.cuda.current_stream()
    g.query_seqs(offsets, chars, out=out, nkmers=nk)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        g.query_seqs(offsets, chars, out=out, nkmers=nk)
        e.record(stream)
        e.synchronize()
        best = min(best, s.elapsed_time(e) / 1e3)
    return best


def capture_query_seqs(g: rb.Rambo, offsets, chars, out, nk):
    """A hipGraph (torch.cuda.CUDAGraph) of one batched rambo_query_seqs call
    with the current query policy: the launches of the batch recorded once
    and replayed as one unit.  The call is made once first, so that the
    library's per-read state is already large enough (nothing is allocated
    while recording)."""
    g.query_seqs(offsets, chars, out=out, nkmers=nk)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.query_seqs(offsets, chars, out=out, nkmers=nk)
    torch.cuda.synchronize()
    return graph


def capture(fn):
    """A hipGraph (torch.cuda.CUDAGraph) of fn(), a sequence of library calls
    on torch's current stream (inserts, clears, queries).  fn runs once
    eagerly first, so that scratch and per-read state already have their size
    (nothing is allocated while recording); inserts are idempotent, so the
    extra eager run changes no answer."""
    fn()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    torch.cuda.synchronize()
    return graph


def time_graph(graph, reps: int = 3) -> float:
    """Best of reps, in seconds, of one replay."""
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        graph.replay()
        e.record(stream)
        e.synchronize()
        best = min(best, s.elapsed_time(e) / 1e3)
    return best


def tune_query_seqs(g: rb.Rambo, offsets, chars, tag: str = "reads", use_cache: bool = True):
    """Pick and apply the fastest queue shape for this batch kind.  Returns a
    dict with the choice, its time and the sweep."""
    key = _key(g, tag)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        g.set_query_policy(c["mode"], c["chunk"], c["waves_per_cu"])
        return dict(c, cached=True)
    n = offsets.numel() - 1
    out = torch.empty((n, g.W), dtype=torch.int32, device=offsets.device)
    nk = torch.empty(n, dtype=torch.int32, device=offsets.device)
    ref = None
    sweep = []
    best = None
    cands = [(rb.QUERY_WAVE_PER_READ, 0, 0)] + [(rb.QUERY_QUEUE, c, w) for c in CHUNKS for w in WAVES_PER_CU]
    for mode, chunk, wpc in cands:
        g.set_query_policy(mode, chunk, wpc)
        t = time_query_seqs(g, offsets, chars, out, nk)
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError("tile shape %s changed the answers" % ((mode, chunk, wpc),))
        sweep.append({"mode": mode, "chunk": chunk, "waves_per_cu": wpc, "seconds": t})
        if best is None or t < best["seconds"]:
            best = sweep[-1]
    g.set_query_policy(best["mode"], best["chunk"], best["waves_per_cu"])
    choice = dict(best)
    cache[key] = choice
    if use_cache:
        _store(cache)
    return dict(choice, cached=False, sweep=sweep)
