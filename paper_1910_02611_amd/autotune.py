"""Tile autotuner for the batched query launches and the partitioned insert.

Queries: sweeps the work-queue shape of rambo_query_seqs (bytes per work
item, persistent waves per compute unit) on a representative batch.
Inserts: tunes the partitioned insert's tile shapes (rambo_set_insert_tiles:
stage-A steps per round, stage-B tile, groups of coarse buckets of stages B
and C, regions per coarse bucket) one at a time from the automatic choice,
on the real insert.  Every candidate is timed with HIP events on the current
stream, the fastest is kept and cached in a JSON file keyed by device, index
shape and workload tag, so a later run starts from it.  Every candidate
computes the same answers or index bits; the sweeps check that too.
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
    return "%s|%d CUs|K%d-B%d-R%d-e%d-m%d|%s" % (getattr(dev, "gcnArchName", ""), dev.multi_processor_count, g.K,
                                                g.B, g.R, g.eta, g.m, tag)


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


def index_digest(g: rb.Rambo, samples: int = 64, words: int = 4096):
    """Per-cell set-bit counts and `samples` spread chunks of index words: a
    cheap stand-in for the whole index when comparing two inserts."""
    fills = g.fill_counts().cpu()
    total = g.index_bytes // 4
    step = max(words, total // samples)
    chunks = [g.index_words(o, min(words, total - o)).cpu() for o in range(0, total, step)]
    return fills, torch.cat(chunks)


def time_insert(g: rb.Rambo, insert, reps: int = 2) -> float:
    """Best of reps, in seconds, of clear + insert() on torch's current stream
    (the clear is outside the timed region).  One untimed insert comes first:
    a change of tile shapes releases the insert's scratch, and the insert
    after it allocates that again."""
    stream = torch.cuda.current_stream()
    g.clear()
    insert()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        g.clear()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        insert()
        e.record(stream)
        e.synchronize()
        best = min(best, s.elapsed_time(e) / 1e3)
    return best


INSERT_KNOBS = {
    "steps": (1, 2),
    "stage_b_tile": (8192, 16384, 32768),
    "groups": (1, 2, 4, 8),
}


def tune_insert(g: rb.Rambo, insert, tag: str, use_cache: bool = True, reps: int = 2, fine_bits_span: int = 1,
                min_gain: float = 0.02):
    """Pick and apply the fastest tile shapes of the partitioned insert for
    this workload: start from the automatic shapes, then try the values of
    one knob at a time (steps, stage-B tile, regions per coarse bucket
    within fine_bits_span of the automatic value, groups), keeping a value
    when it is faster by more than min_gain (so that timing noise does not
    flip the choice).  insert() must insert the workload into g (cleared
    before each timing).  Returns the choice, its time and the sweep."""
    key = _key(g, "insert|" + tag)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        g.set_insert_tiles(**c["tiles"])
        return dict(c, cached=True)
    g.set_insert_tiles()
    base = g.insert_tiles()
    cur = {"steps": 0, "stage_b_tile": 0, "groups": 0, "fine_bits": 0}
    best_t = time_insert(g, insert, reps)
    ref = index_digest(g)
    sweep = [{"tiles": dict(cur), "effective": g.insert_tiles(), "seconds": best_t}]
    knobs = dict(INSERT_KNOBS)
    knobs["fine_bits"] = tuple(f for f in range(base["fine_bits"] - fine_bits_span, base["fine_bits"] + fine_bits_span + 1)
                               if 8 <= f <= 12)
    # shapes already timed, as the library resolves them (the groups that
    # an automatic choice resolves to are known once an insert has run)
    def resolved(tiles, eff):
        return (eff["steps"], eff["stage_b_tile"], eff["fine_bits"], tiles["groups"] or auto_groups[eff["fine_bits"]])

    auto_groups = {base["fine_bits"]: sweep[0]["effective"]["groups"]}
    seen = {resolved(cur, sweep[0]["effective"])}
    for name in ("steps", "stage_b_tile", "fine_bits", "groups"):
        for v in knobs[name]:
            trial = dict(cur, **{name: v})
            try:
                g.set_insert_tiles(**trial)
            except rb.RamboError:
                continue   # not possible for this index (LDS or bucket limits)
            eff = g.insert_tiles()
            if trial["groups"] == 0 and eff["fine_bits"] not in auto_groups:
                auto_groups[eff["fine_bits"]] = -eff["fine_bits"]   # not known yet: a shape of its own
            shape = resolved(trial, eff)
            if shape in seen:
                continue
            seen.add(shape)
            t = time_insert(g, insert, reps)
            fills, words = index_digest(g)
            if not (torch.equal(fills, ref[0]) and torch.equal(words, ref[1])):
                raise RuntimeError("insert tiles %s changed the index" % trial)
            sweep.append({"tiles": dict(trial), "effective": g.insert_tiles(), "seconds": t})
            if trial["groups"] == 0:
                auto_groups[sweep[-1]["effective"]["fine_bits"]] = sweep[-1]["effective"]["groups"]
            if t < best_t * (1.0 - min_gain):
                best_t, cur = t, trial
    g.set_insert_tiles(**cur)
    choice = {"tiles": cur, "effective": g.insert_tiles(), "seconds": best_t, "automatic": base,
              "automatic_seconds": sweep[0]["seconds"]}
    cache[key] = choice
    if use_cache:
        _store(cache)
    return dict(choice, cached=False, sweep=sweep)
