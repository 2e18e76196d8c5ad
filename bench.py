#!/usr/bin/env python3
"""RAMBO on one MI355X: bulk insertion, batched queries and served requests.

Headline workload ("large", the largest configuration that fits one GPU):
K = 100 000 genome sets, lognormal lengths (median 100 kbp, 10 kbp - 1 Mbp)
cut from 5 000 random 1 Mbp ancestors with 1% substitutions (~1.3e10
31-mers); index B = 1 000, R = 6, m = 2^27 bits per cell, eta = 2 (96 GiB
bit-sliced); 1e6 reads of 150 bp (80% set substrings with 1% further
substitutions, 20% random), each answered as the ascending list of the
sets that hold all of its 31-mers.

One step = zero the index + insert every set (partitioned insert, in as
many scratch batches as the insert needs) + answer every read
(rambo_query_seqs_ids, called asynchronously into buffers sized beforehand;
its overflow status is checked after the timed steps).  Inputs are resident
in device memory before timing.  Before the first insert the large section
also measures the insert's stage-A write pattern alone
(rambo_roofline_append) and reports stage A against it.
`value` is k-mer queries per second of the query phase (every valid 31-mer
window of the reads is one k-mer query answered); inserts per second of the
insert phase are reported beside it.  Phase times come from HIP events on
the stream the kernels run on; per-kernel times from events the library
records around each launch on that stream.

Further sections of the same JSON line: `served` (K = 10 000, B = 200,
R = 5, m = 2^29: an 80 GiB index; insert, then the query server under
Poisson load at 8 points from 10% to 120% of its saturated rate, p50/p99 in
`latency`), `mid` (K = 1 000, B = 50, R = 4, m = 2^28; 1e7 single k-mer
queries, the one-launch-per-query comparator, ceilings measured over an
index-sized buffer, folding over), `tiny` (K = 64, B = 8, R = 3, m = 2^18;
1e4 k-mer queries, with the oracle timed on the whole workload),
`batched_reads` (1e5 reads of 100 - 10 000 bp on the tiny index, one
persistent launch, graph replay, the oracle on a sample), `documents` (the
word-unigram index on raw 64-bit keys) and `cpu_baseline` (the oracle on a
bounded sample of the headline workload).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
SECTOR = 64             # bytes of one random row access at HBM (one sector)
METRIC = "k-mer queries/s and inserts/s on 1 GPU (% of random-HBM roofline); p50/p99 latency"
SECTIONS = ("large", "served", "mid", "tiny", "batched", "documents")
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a, view):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(view)).to("cuda")


def n_windows(sets, k: int) -> int:
    return int(np.sum(np.maximum(sets.lengths().astype(np.int64) - k + 1, 0)))


# ------------------------------------------------------------------ rooflines

def measured_traffic(names: dict, workload: str) -> dict:
    """HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE) from the
    committed rocprofv3 summary of one workload, for stage name -> kernel
    name as profiled; empty when the summary is missing or the kernel sources
    changed since it was taken."""
    from paper_1910_02611_amd.profsum import load_traffic
    t = load_traffic(os.path.join(PROFILES, "traffic_%s.json" % workload))
    if t is None:
        return {}
    out = {}
    for stage, k in names.items():   # a kernel name, or the start of one (template arguments)
        hit = [n for n in t["kernels"] if n == k or n.startswith(k)]
        if hit:
            out[stage] = t["kernels"][hit[0]]["bytes"]
    return out


def hbm_entry(kernel, bytes_per_launch, ms_per_launch, what, traffic=None, launches=1):
    gbs = bytes_per_launch / (ms_per_launch / 1e3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "ms": ms_per_launch, "launches": launches,
            "work_per_launch": bytes_per_launch, "work": what}


def insert_rooflines(kernels: dict, n_win: int, n_bases: int, R: int, eta: int, index_bytes: int,
                     fresh_first: bool, workload: str, code_input: bool = False) -> list:
    """Roofline entries of the partitioned insert's kernels, per launch
    (each scratch batch launches stages A, B and C once).  Algorithmic bytes
    follow the partitioned streaming bound of the insert: every bit target
    is an 8-byte record written once by the binning and read once by the
    apply, the index is read and written once, the input is read once.
    Stage A is charged the record writes (8 B per target) and the input
    (1 B per base, or 8 B per code); stage C the record reads (8 B per
    target) and the index (written once per batch, and read back except in
    a first batch into an all-zero index).  Stage B, the second partition
    pass, is this design's own cost and is charged the 4-byte records it
    moves (read and written once).  `insert_pipeline` sets the whole insert
    against the bound itself (2 x index + 16 B per target + input)."""
    RE = R * eta
    targets = n_win * RE
    a_name = "k_bin_codes" if code_input else ("k_bin_pieces" if "k_bin_pieces" in kernels else "k_bin_windows")
    stage_k = {a_name: "%s_hold<%d, %d>" % (a_name, R, eta), "k_bin_regions": "k_bin_regions",
               "k_apply_regions": "k_apply_regions"}
    if a_name == "k_bin_pieces":
        stage_k[a_name] = "k_bin_pieces<%d, %d" % (R, eta)
    # one stage-A launch per scratch batch; stages B and C launch once per
    # group of coarse buckets in each batch
    batches = kernels[a_name][1] if a_name in kernels else 1
    tr = measured_traffic(stage_k, workload)
    out = []
    if a_name in kernels:
        ms, calls = kernels[a_name]
        byts = (targets * 8 + (n_win * 8 if code_input else n_bases)) / calls
        out.append(hbm_entry(a_name, byts, ms / calls, "8 B record per bit target written + input read once "
                             "(partitioned bound's share of stage A)", tr.get(a_name), calls))
    if "k_bin_regions" in kernels:
        ms, calls = kernels["k_bin_regions"]
        out.append(hbm_entry("k_bin_regions", targets * 8 / calls, ms / calls,
                             "4 B record per bit target read + written (the second partition pass)",
                             tr.get("k_bin_regions"), calls))
    if "k_apply_regions" in kernels:
        ms, calls = kernels["k_apply_regions"]
        idx = index_bytes * (2 * batches - (1 if fresh_first else 0))
        out.append(hbm_entry("k_apply_regions", (targets * 8 + idx) / calls, ms / calls,
                             "8 B record per bit target read + index written once per batch (and read back "
                             "unless the index was all zero); a launch covers one group of regions",
                             tr.get("k_apply_regions"), calls))
    total_ms = sum(kernels[k][0] for k in (a_name, "k_bin_regions", "k_apply_regions", "k_zero_u32")
                   if k in kernels)
    if total_ms > 0:
        byts = 2 * index_bytes + 16 * targets + (n_win * 8 if code_input else n_bases)
        e = hbm_entry("insert_pipeline", byts, total_ms, "partitioned bound of the whole insert: index read + "
                      "written once, 16 B per bit target, input once")
        e["batches"] = batches
        e["groups_per_batch"] = kernels.get("k_bin_regions", (0, batches))[1] // max(1, batches)
        out.append(e)
    return out


def query_kmers_roofline(kernels, n_q, R, eta, S, W, workload):
    if "k_query_kmers" not in kernels:
        return None
    ms, calls = kernels["k_query_kmers"]
    SW = max(1, S // 32)
    byts = n_q * (R * eta * max(SECTOR, S // 8) + 4 * W + 8) / calls
    tr = measured_traffic({"q": "k_query_kmers<%d, %d, %d>" % (SW, R, eta)}, workload).get("q")
    return hbm_entry("k_query_kmers", byts, ms / calls, "R*eta row sectors + K-bit answer + code per query", tr,
                     calls)


def tune_insert(g, insert, tag: str, args, reps: int = 2) -> dict | None:
    """The insert autotuner's pick for this workload (applied to g), or None
    with --no-tune-insert."""
    if args.no_tune_insert:
        return None
    from paper_1910_02611_amd import autotune
    t = time.time()
    r = autotune.tune_insert(g, insert, tag, reps=reps)
    log("%s: insert tiles %s (automatic %s): %.1f ms vs %.1f ms automatic (%s, %.1f s)"
        % (tag, r["effective"], r["automatic"], r["seconds"] * 1e3, r["automatic_seconds"] * 1e3,
           "from the tuning cache" if r["cached"] else "%d shapes timed" % len(r["sweep"]), time.time() - t))
    return r


def time_insert_graph(g, insert, reps: int = 3) -> dict:
    """clear + insert recorded as one hipGraph and replayed, against the
    eager calls: best replay time, and whether the replayed index equals the
    eager one (digest of per-cell fills and sampled words)."""
    import torch
    from paper_1910_02611_amd import autotune
    g.clear()
    insert()
    torch.cuda.synchronize()
    ref = autotune.index_digest(g)

    def step():
        g.clear()
        insert()

    graph = autotune.capture(step)
    t = autotune.time_graph(graph, reps)
    got = autotune.index_digest(g)
    same = bool(torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1]))
    del graph
    return {"replay_ms": t * 1e3, "identical": same}


# ------------------------------------------------------------------ timing

def time_steps(g, insert, query, steps: int, warmup: int):
    """`warmup` untimed then `steps` timed steps of clear + insert + query on
    torch's current stream.  Returns wall seconds of the timed steps, mean
    phase milliseconds and per-kernel (total ms per step, launches per step)."""
    import torch
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]

    def one_step(e=None):
        if e: e[0].record(stream)
        g.clear()
        if e: e[1].record(stream)
        insert()
        if e: e[2].record(stream)
        query()
        if e: e[3].record(stream)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    g.stage_times()        # drop anything recorded so far
    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        one_step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.set_timing(False)
    kernels = {k: (v[0] / steps, max(1, v[1] // steps)) for k, v in g.stage_times(calls=True).items()}
    phases = {name: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in ev]))
              for i, name in enumerate(("clear", "insert", "query"))}
    return wall, phases, kernels


def log_rooflines(roofs):
    for r in roofs:
        if r:
            log("  %-18s %9.3f ms x%-3d %-4s %8.4g %s (%.1f%% of %g)" % (
                r["kernel"], r["ms"], r.get("launches", 1), r["bound"], r["achieved"], r["unit"], 100 * r["frac"],
                r["peak"]))


# ------------------------------------------------------------------ sections

def section_large(args):
    """The headline: the 96 GiB index, 1e6 150-bp reads as ID lists."""
    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo
    cfg = synth.INDEX_LARGE
    t = time.time()
    sets = synth.config_large()
    rd = synth.reads(3205, sets, args.large_reads, median_len=150, min_len=150, max_len=150, substr_frac=0.8,
                     read_sub_rate=0.01)
    n_win = n_windows(sets, cfg["k"])
    log("large: %d sets, %d bases (%d windows), %d reads (%.1f s to generate)"
        % (sets.n, sets.chars.size, n_win, rd.n, time.time() - t))
    g = Rambo(**cfg, seed=2005)
    if args.insert_policy:
        g.set_insert_policy(args.insert_policy)
    dsets = (to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    n_bases = int(sets.chars.size)
    n_sets = sets.n
    off, ch = to_dev(rd.offsets, np.int64), to_dev(rd.chars, np.uint8)
    ids = torch.empty(16 << 20, dtype=torch.int32, device="cuda")
    nk = torch.empty(rd.n, dtype=torch.int32, device="cuda")
    id_offsets = torch.empty(rd.n + 1, dtype=torch.int64, device="cuda")
    state = {}

    def query():
        # asynchronous: every kernel of the ID-list query runs in the timed
        # phase; the overflow status is checked once the steps are done
        state["r"] = g.query_seqs_ids(off, ch, ids=ids, nkmers=nk, id_offsets=id_offsets, wait=False)

    pattern = stage_a_write_pattern(g) if not args.no_measured_ceilings else None
    tuning = tune_insert(g, lambda: g.insert_seqs(*dsets), "large", args, reps=1)
    wall, ph, kernels = time_steps(g, lambda: g.insert_seqs(*dsets), query, args.steps, args.warmup)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (large): an ID list did not fit, or a bad input")
    id_off, got_ids, nkm = state["r"]
    got_ids = got_ids[:int(id_off[-1].item())]
    kmers = int(nkm.to(torch.int64).sum())
    sizes = np.diff(id_off.cpu().numpy())
    RE = cfg["R"] * cfg["eta"]
    roofs = insert_rooflines(kernels, n_win, n_bases, cfg["R"], cfg["eta"], g.index_bytes, True, "large")
    if "k_query_seqs" in kernels:
        # reads with a non-empty answer probe every window in every
        # repetition: R*eta rows of S/8 = 128 bytes each (one line); reads
        # cut short by the early exit are not credited
        ms, calls = kernels["k_query_seqs"]
        full = int(nkm.cpu().numpy().astype(np.int64)[sizes > 0].sum())
        tr = measured_traffic({"q": "k_query_seqs<"}, "large").get("q")
        roofs.append(hbm_entry("k_query_seqs", full * RE * max(SECTOR, g.row_bits // 8) / calls, ms / calls,
                               "R*eta rows of max(64, S/8) bytes per window of the reads with a non-empty answer "
                               "(the early exit is not credited)", tr, calls))
    if pattern is not None and "k_bin_pieces" in kernels:
        ms, calls = kernels["k_bin_pieces"]
        ent = n_win * RE * 4 / calls / (ms / calls / 1e3) / 1e9
        pattern["stage_a_entries_GBps"] = ent
        pattern["stage_a_frac_of_misaligned"] = ent / pattern["misaligned"]["GBps"]
        log("large: stage A writes its 4-byte entries at %.0f GB/s: %.0f%% of the %.0f GB/s its write pattern "
            "sustains alone (%.0f GB/s with aligned runs)" % (ent, 100 * pattern["stage_a_frac_of_misaligned"],
                                                              pattern["misaligned"]["GBps"],
                                                              pattern["aligned"]["GBps"]))
    res = {
        "workload": "large: K=100000 genome sets (~1.3e10 31-mers), B=1000, R=6, m=2^27, eta=2 (96 GiB); "
                    "%d reads of 150 bp (80%% set substrings with 1%% substitutions) as set-ID lists" % rd.n,
        "K": cfg["K"], "B": cfg["B"], "R": cfg["R"], "m": cfg["m"], "eta": cfg["eta"], "k": cfg["k"],
        "sets": n_sets, "bases": n_bases, "inserts": n_win, "bit_targets": n_win * RE, "reads": rd.n,
        "read_kmers": kmers, "index_bytes": g.index_bytes,
        "phase_ms": ph, "ms_per_step": wall / args.steps * 1e3,
        "inserts_per_s": n_win / (ph["insert"] / 1e3),
        "k_mer_queries_per_s": kmers / (ph["query"] / 1e3),
        "reads_per_s": rd.n / (ph["query"] / 1e3),
        "kernel_ms": {k: v[0] for k, v in kernels.items()},
        "kernel_launches": {k: v[1] for k, v in kernels.items()},
        "rooflines": sorted(roofs, key=lambda r: -r["ms"] * r.get("launches", 1)),
        "answer_sets_hist_0_to_10plus": np.bincount(np.minimum(sizes, 10), minlength=11).tolist(),
        "insert_tuning": tuning,
        "stage_a_write_pattern": pattern,
    }
    log("large: step %.1f ms: clear %.2f, insert %.1f ms (%.3g inserts/s), ID-list query %.2f ms (%.3g k-mer "
        "queries/s, %.3g reads/s)" % (res["ms_per_step"], ph["clear"], ph["insert"], res["inserts_per_s"],
                                      ph["query"], res["k_mer_queries_per_s"], res["reads_per_s"]))
    log_rooflines(res["rooflines"])
    g.close()
    del dsets, off, ch, ids, nk, state
    torch.cuda.empty_cache()
    return res, sets, rd


def section_served(args):
    """The 80 GiB index: insert, then the query server under Poisson load."""
    import torch
    from paper_1910_02611_amd import serve, synth
    from paper_1910_02611_amd.rambo import Rambo, Server
    cfg = synth.INDEX_SERVED
    t = time.time()
    sets = synth.config_served()
    batch = synth.served_requests(4004, sets, args.serve_requests)
    reqs = serve.split_requests(batch)
    n_win = n_windows(sets, cfg["k"])
    log("served: %d sets, %d bases, %d requests of %d reads (%.1f s to generate)"
        % (sets.n, sets.chars.size, len(reqs), batch.n, time.time() - t))
    g = Rambo(**cfg, seed=2004)
    if args.insert_policy:
        g.set_insert_policy(args.insert_policy)
    dsets = (to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    torch.cuda.synchronize()
    wall, ph, kernels = time_steps(g, lambda: g.insert_seqs(*dsets), lambda: None, 1, 1)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (served)")
    del dsets
    torch.cuda.empty_cache()
    roofs = insert_rooflines(kernels, n_win, int(sets.chars.size), cfg["R"], cfg["eta"], g.index_bytes, True,
                             "served")
    log("served: insert %.1f ms (%.3g inserts/s)" % (ph["insert"], n_win / (ph["insert"] / 1e3)))
    log_rooflines(roofs)
    loads = [float(x) for x in args.serve_loads.split(",")]
    with Server(g, max_slots=args.serve_slots, use_graphs=args.serve_graphs) as srv:
        serve.saturated(srv, reqs[: min(300, len(reqs))], g.W)   # warm-up
        res = serve.sweep_native(srv, batch, loads)
        # answers in the mix equal the same requests answered alone
        sample = reqs[:200]
        sids = [srv.submit(o, c) for o, c in sample]
        mixed = [srv.wait(i, len(o) - 1)[0] for i, (o, _) in zip(sids, sample)]
        res["server"] = srv.stats()
    # (alone, on the index as it was in the mix: before the streaming inserts)
    same = True
    for (o, c), got in zip(sample, mixed):
        alone, _ = g.query_seqs(to_dev(o, np.int64), to_dev(c, np.uint8))
        same = same and bool(np.array_equal(alone.cpu().numpy().view(np.uint32), got))
    with Server(g, max_slots=args.serve_slots, use_graphs=args.serve_graphs) as srv:
        # streaming inserts among the queries at a quarter of the saturated
        # rate (Python driver): the same arrivals with and without them
        rate = 0.25 * res["saturated"]["qps"]
        n_ins_req = min(len(reqs), 4000)
        arr = synth.poisson_arrivals(5100, n_ins_req, rate)
        ins = serve.insert_stream(5101, sets, max(1, int(arr[-1] / 0.02)), 0.02, 32, 5000)
        plain = serve.run_open_loop(srv, reqs[:n_ins_req], arr, g.W)
        with_ins = serve.run_open_loop(srv, reqs[:n_ins_req], arr, g.W, inserts=ins)
    sat = res["saturated"]
    log("served: saturated %.4g requests/s (%.4g reads/s)" % (sat["qps"], sat["reads_per_s"]))
    for p in res["points"]:
        log("  load %.2f: offered %.4g/s achieved %.4g/s  p50 %.3f ms  p99 %.3f ms (host queue p99 %.3f, "
            "service p99 %.3f; cgroup CPU throttling %s; worker max loop gap %.0f us, enqueue %.0f us, "
            "query %.0f us)"
            % (p["load"], p["offered_qps"], p["qps"], p["p50_ms"], p["p99_ms"], p["queue_p99_ms"],
               p["service_p99_ms"], "%d periods, %.1f ms" % (p["cpu_throttled_periods"], p["cpu_throttled_ms"])
               if "cpu_throttled_ms" in p else "n/a", p["worker_max_loop_gap_us"], p["worker_max_enqueue_us"],
               p["worker_max_query_us"]))
    log("served: 200 requests alone == in the mix: %s; with %d streaming inserts at 25%% load: query p50 %.3f "
        "p99 %.3f ms (without: %.3f / %.3f)" % (same, with_ins["inserts"], with_ins["p50_ms"], with_ins["p99_ms"],
                                                plain["p50_ms"], plain["p99_ms"]))
    keep = ("load", "offered_qps", "qps", "reads_per_s", "p50_ms", "p99_ms", "mean_ms", "queue_p50_ms",
            "queue_p99_ms", "service_p99_ms", "cpu_throttled_periods", "cpu_throttled_ms", "worker_max_loop_gap_us",
            "worker_max_enqueue_us", "worker_max_query_us")
    out = {
        "workload": "served: K=10000 genome sets (~6.6e9 31-mers), B=200, R=5, m=2^29, eta=2 (80 GiB); requests "
                    "of U{1..64} reads, log-uniform 150-5000 bp, 70%% set substrings; %d requests per load point, "
                    "Poisson arrivals, native open-loop driver, %d slots, %s" % (
                        len(reqs), args.serve_slots,
                        "fixed slot buffers, graph replay" if args.serve_graphs else
                        "batches admitted by device bytes from a 1 GiB pool"),
        "K": cfg["K"], "B": cfg["B"], "R": cfg["R"], "m": cfg["m"], "eta": cfg["eta"],
        "inserts": n_win, "index_bytes": g.index_bytes,
        "insert_ms": ph["insert"], "inserts_per_s": n_win / (ph["insert"] / 1e3),
        "kernel_ms": {k: v[0] for k, v in kernels.items()},
        "kernel_launches": {k: v[1] for k, v in kernels.items()},
        "rooflines": sorted(roofs, key=lambda r: -r["ms"] * r.get("launches", 1)),
        "saturated": {k: sat[k] for k in ("qps", "reads_per_s", "p50_ms", "p99_ms")},
        "points": [{k: p[k] for k in keep if k in p} for p in res["points"]],
        "alone_equals_mixed": {"requests": len(sample), "identical": same},
        "with_inserts": dict({k: with_ins[k] for k in ("qps", "p50_ms", "p99_ms", "inserts", "insert_bases",
                                                       "insert_p50_ms", "insert_p99_ms")},
                             load=0.25, requests=n_ins_req,
                             without_inserts={k: plain[k] for k in ("qps", "p50_ms", "p99_ms")}),
        "server": res["server"],
    }
    g.close()
    del sets, batch, reqs
    torch.cuda.empty_cache()
    return out


def section_mid(args):
    """K = 1 000 sets, 8 GiB index, 1e7 single k-mer queries."""
    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo
    cfg = synth.INDEX_MID
    t = time.time()
    sets = synth.config_mid()
    q = synth.kmer_queries(3002, sets, args.queries, 31)
    n_win = n_windows(sets, cfg["k"])
    log("mid: %d sets, %d bases, %d queries (%.1f s to generate)" % (sets.n, sets.chars.size, q.n, time.time() - t))
    g = Rambo(**cfg, seed=2002)
    if args.insert_policy:
        g.set_insert_policy(args.insert_policy)
    dsets = (to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    qoff, qchars = to_dev(q.offsets, np.int64), to_dev(q.chars, np.uint8)
    codes = g.extract_kmers(qoff, qchars)[qoff[:-1]].contiguous()
    del qchars
    out = torch.empty((q.n, g.W), dtype=torch.int32, device="cuda")
    tuning = tune_insert(g, lambda: g.insert_seqs(*dsets), "mid", args)
    wall, ph, kernels = time_steps(g, lambda: g.insert_seqs(*dsets), lambda: g.query_kmers(codes, out=out),
                                   args.steps, args.warmup)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (mid)")
    R, eta, S, W = cfg["R"], cfg["eta"], g.row_bits, g.W
    roofs = insert_rooflines(kernels, n_win, int(sets.chars.size), R, eta, g.index_bytes, True, "mid")
    qr = query_kmers_roofline(kernels, q.n, R, eta, S, W, "mid")
    roofs = sorted(roofs + [qr], key=lambda r: -r["ms"] * r.get("launches", 1))
    res = {
        "workload": "mid: K=1000 genome sets (~2.5e8 31-mers), B=50, R=4, m=2^28, eta=2 (8 GiB); 1e7 single 31-mer "
                    "queries (50% present)",
        "K": cfg["K"], "B": cfg["B"], "R": R, "m": cfg["m"], "eta": eta, "inserts": n_win, "queries": q.n,
        "phase_ms": ph, "ms_per_step": wall / args.steps * 1e3,
        "inserts_per_s": n_win / (ph["insert"] / 1e3), "k_mer_queries_per_s": q.n / (ph["query"] / 1e3),
        "kernel_ms": {k: v[0] for k, v in kernels.items()},
        "rooflines": roofs,
        "insert_tuning": tuning,
    }
    log("mid: step %.2f ms: insert %.2f ms (%.3g inserts/s), query %.3f ms (%.3g queries/s)"
        % (res["ms_per_step"], ph["insert"], res["inserts_per_s"], ph["query"], res["k_mer_queries_per_s"]))
    log_rooflines(roofs)
    res["insert_graph"] = time_insert_graph(g, lambda: g.insert_seqs(*dsets))
    log("mid: clear + insert as one captured graph: %.2f ms per replay (eager insert %.2f ms), index identical %s"
        % (res["insert_graph"]["replay_ms"], ph["insert"], res["insert_graph"]["identical"]))
    if not args.no_measured_ceilings:
        res["measured_ceilings"] = measured_ceilings(g.index_bytes, S, R * eta, res["k_mer_queries_per_s"],
                                                     kernels)
    if args.plain_prefix > 0:
        rate, same = plain_path(g, codes, out, min(args.plain_prefix, q.n))
        res["plain_path"] = {"k_mer_queries_per_s": rate, "prefix": min(args.plain_prefix, q.n), "identical": same,
                             "speedup_batched": res["k_mer_queries_per_s"] / rate}
        log("mid: plain one-launch-per-query path %.3g queries/s on %d, identical=%s"
            % (rate, args.plain_prefix, same))
    res["skewed_reads"] = skewed_reads(g, sets)
    if not args.no_fold:
        res["fold"] = fold_timing(g)
    g.close()
    del out, codes, dsets
    torch.cuda.empty_cache()
    return res


def skewed_reads(g, sets, n_short: int = 20000, n_long: int = 16, long_len: int = 500_000) -> dict:
    """A batch where one wave per read is unbalanced: n_short 150-bp reads
    and n_long exact substrings of long_len bases (every window of these
    hits, so no early exit).  The query autotuner sweeps both schedules;
    the work queue splits the long reads into chunks that many waves take."""
    import torch
    from paper_1910_02611_amd import autotune, synth
    from paper_1910_02611_amd.rambo import QUERY_QUEUE, QUERY_WAVE_PER_READ
    lens = np.concatenate([np.full(n_short, 150), np.full(n_long, long_len)])
    np.random.default_rng(1).shuffle(lens)
    rd = synth.reads(3060, sets, lens.size, median_len=0, min_len=150, max_len=long_len, substr_frac=1.0,
                     lengths=lens)
    off, ch = to_dev(rd.offsets, np.int64), to_dev(rd.chars, np.uint8)
    tune = autotune.tune_query_seqs(g, off, ch, tag="skewed-reads", use_cache=False)
    out = torch.empty((rd.n, g.W), dtype=torch.int32, device="cuda")
    nk = torch.empty(rd.n, dtype=torch.int32, device="cuda")
    res = {"reads": rd.n, "long_reads": n_long, "long_len": int(rd.lengths().max()), "bases": int(rd.chars.size),
           "tile": {k: tune[k] for k in ("mode", "chunk", "waves_per_cu")}}
    ref = None
    for name, mode in (("wave_per_read", QUERY_WAVE_PER_READ), ("work_queue", QUERY_QUEUE)):
        g.set_query_policy(mode, tune["chunk"] if mode == QUERY_QUEUE and tune["mode"] == QUERY_QUEUE else 0,
                           tune["waves_per_cu"] if mode == QUERY_QUEUE and tune["mode"] == QUERY_QUEUE else 0)
        tm = autotune.time_query_seqs(g, off, ch, out, nk, reps=3)
        ref = out.clone() if ref is None else ref
        res[name] = {"ms": tm * 1e3, "reads_per_s": rd.n / tm, "identical": bool(torch.equal(out, ref))}
    g.set_query_policy(0)
    log("mid: skewed batch (%d x 150 bp + %d x %d bp): one wave per read %.3f ms, work queue %.3f ms (identical %s);"
        " tuned %s" % (n_short, n_long, long_len, res["wave_per_read"]["ms"], res["work_queue"]["ms"],
                       res["work_queue"]["identical"], res["tile"]))
    return res


REGION_BITS = 20   # the insert's index regions (stage C): 2^20 bits, 128 KiB of LDS


def stage_a_write_pattern(g, gib: float = 8.0) -> dict:
    """The write pattern of the insert's stage A measured alone on this GPU
    (before the first insert allocates its scratch): runs of 16 four-byte
    entries appended to one chunk per (coarse bucket, workgroup), as many
    buckets as this index has and one workgroup per CU, with runs starting
    inside 64-byte segments (as the binning's running cursors do) and, for
    reference, aligned to them."""
    import torch
    from paper_1910_02611_amd import roofline
    fb = g.insert_tiles()["fine_bits"]
    streams = -(-g.index_bytes * 8 // (1 << (REGION_BITS + fb)))
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    out = roofline.append(int(gib * 2**30), streams, 16, cus)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()   # the probe's buffer must not shrink the insert's scratch
    return out


def measured_ceilings(index_bytes: int, S: int, RE: int, q_per_s: float, kernels: dict) -> dict:
    """Ceilings measured on this GPU over a buffer as large as the index (so
    TLB and last-level-cache effects are included): random gathers of one
    row (S/8 bytes, at least 4) against the k-mer queries, counting the rows
    each query issues as R*eta (the early exit is not subtracted); a
    streaming copy against the partitioned insert's streaming stages."""
    from paper_1910_02611_amd import roofline
    G = max(4, S // 8)
    m = roofline.measure(index_bytes, n_access=1 << 27, sizes=(G,))
    gathers = m["gather"][str(G)]["accesses_per_s"]
    copy = m["copy"]["GBps_read_plus_write"] * 1e9
    log("mid: measured over %.1f GiB: random %d-byte gathers %.3g/s, streaming copy %.0f GB/s (read + write)"
        % (index_bytes / 2**30, G, gathers, copy / 1e9))
    out = {"buffer_bytes": index_bytes,
           "query": {"achieved": q_per_s * RE, "ceiling": gathers, "unit": "row gathers/s",
                     "frac": q_per_s * RE / gathers, "row_bytes": G},
           "random_atomic_or_per_s": m["atomic_or"]["accesses_per_s"],
           "streaming_copy_bytes_per_s": copy}
    return out


def plain_path(g, codes, out_batched, n_prefix: int):
    """The one-launch-per-query GPU path on a prefix, with identical answers."""
    import torch
    pre = codes[:n_prefix].contiguous()
    g.query_kmers(pre, plain=True)   # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = g.query_kmers(pre, plain=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return n_prefix / dt, bool(torch.equal(got, out_batched[:n_prefix]))


def fold_timing(g):
    """Folding over the resident index once (B -> B/2): the k_fold kernel's
    duration against reading the old index and writing the new one once,
    and the whole call (tables rebuilt on the host included)."""
    old_bytes, B = g.index_bytes, g.B
    g.set_timing(True)
    g.stage_times()
    t0 = time.perf_counter()
    g.fold()
    wall = time.perf_counter() - t0
    ms = g.stage_times()["k_fold"]
    g.set_timing(False)
    moved = old_bytes + g.index_bytes
    kname = {32: "k_fold_narrow<1>", 64: "k_fold_narrow<2>"}.get(g.row_bits, "k_fold")
    e = hbm_entry(kname, moved, ms, "old index read once + folded index written once",
                  measured_traffic({"k_fold": kname}, "mid").get("k_fold"))
    log("mid: fold B %d -> %d: %s %.3f ms (%.0f GB/s, %.1f%% of HBM peak), call %.1f ms"
        % (B, g.B, kname, ms, e["achieved"], 100 * e["frac"], wall * 1e3))
    return {"B_from": B, "B_to": g.B, "index_bytes_from": old_bytes, "index_bytes_to": g.index_bytes,
            "call_ms": wall * 1e3, "roofline": e}


def section_tiny(args):
    """K = 64 sets, 768 KiB index, 1e4 single k-mer queries; the oracle
    builds the same index and answers the same queries on the host."""
    import oracle
    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    q = synth.kmer_queries(3001, sets, 10_000, 31)
    n_win = n_windows(sets, cfg["k"])
    g = Rambo(**cfg, seed=2001)
    dsets = (to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    qoff, qchars = to_dev(q.offsets, np.int64), to_dev(q.chars, np.uint8)
    codes = g.extract_kmers(qoff, qchars)[qoff[:-1]].contiguous()
    out = torch.empty((q.n, g.W), dtype=torch.int32, device="cuda")
    wall, ph, kernels = time_steps(g, lambda: g.insert_seqs(*dsets), lambda: g.query_kmers(codes, out=out),
                                   max(args.steps, 20), args.warmup)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (tiny)")
    got = out.cpu().numpy().view(np.uint32)
    g.close()
    # the oracle on the whole workload, on the host's threads
    nthreads = host_threads()
    ocodes = oracle.extract(q.offsets, q.chars, cfg["k"])[q.offsets[:-1].astype(np.int64)]
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2001)
    t0 = time.perf_counter()
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, nthreads)
    t_oi = time.perf_counter() - t0
    t0 = time.perf_counter()
    want = o.query_kmers(ocodes, nthreads)
    t_oq = time.perf_counter() - t0
    o.close()
    same = bool(np.array_equal(got, want))
    res = {
        "workload": "tiny: K=64 genome sets (8 ancestors of 5 kbp, 1% substitutions), B=8, R=3, m=2^18, eta=2; "
                    "1e4 single 31-mer queries (50% present)",
        "inserts": n_win, "queries": q.n, "phase_ms": ph, "ms_per_step": wall / max(args.steps, 20) * 1e3,
        "inserts_per_s": n_win / (ph["insert"] / 1e3), "k_mer_queries_per_s": q.n / (ph["query"] / 1e3),
        "kernel_ms": {k: v[0] for k, v in kernels.items()},
        "oracle": {"threads": nthreads, "insert_s": t_oi, "inserts_per_s": n_win / t_oi, "query_s": t_oq,
                   "k_mer_queries_per_s": q.n / t_oq, "answers_identical": same},
    }
    log("tiny: insert %.3f ms (%.3g inserts/s), query %.4f ms (%.3g queries/s); oracle on %d threads: insert "
        "%.3f s, queries %.3f s (%.3g/s), answers identical %s"
        % (ph["insert"], res["inserts_per_s"], ph["query"], res["k_mer_queries_per_s"], nthreads, t_oi, t_oq,
           q.n / t_oq, same))
    return res


def section_batched(args):
    """Batched sequence queries (Sec. 3.2.1) on the tiny index: reads of
    lognormal length (median 1 000, 100-10 000 bp), 70% substrings of a set
    genome.  One launch with the autotuned tile, the same batch as a replayed
    graph, one wave per read, one launch per read; the oracle on a sample."""
    import oracle
    import torch
    from paper_1910_02611_amd import autotune, roofline, synth
    from paper_1910_02611_amd.rambo import Rambo, QUERY_QUEUE, QUERY_WAVE_PER_READ
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    g = Rambo(**cfg, seed=2001)
    g.insert_seqs(to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    t = time.time()
    rd = synth.config_batched_reads(sets, args.reads)
    log("batched: %d reads, %d bases (%.1f s)" % (rd.n, rd.chars.size, time.time() - t))
    off, ch = to_dev(rd.offsets, np.int64), to_dev(rd.chars, np.uint8)
    tune = autotune.tune_query_seqs(g, off, ch, tag="batched-reads", use_cache=False)
    out = torch.empty((rd.n, g.W), dtype=torch.int32, device="cuda")
    nk = torch.empty(rd.n, dtype=torch.int32, device="cuda")
    t_q = autotune.time_query_seqs(g, off, ch, out, nk, reps=5)
    windows = int(nk.to(torch.int64).sum())
    full_windows = int(nk.to(torch.int64)[out.ne(0).any(dim=1)].sum())
    out_g, nk_g = torch.empty_like(out), torch.empty_like(nk)
    graph = autotune.capture_query_seqs(g, off, ch, out_g, nk_g)
    same_g = True
    for _ in range(3):
        out_g.zero_()
        graph.replay()
        g.query_seqs(off, ch, out=out, nkmers=nk)
        torch.cuda.synchronize()
        same_g = same_g and bool(torch.equal(out_g, out)) and bool(torch.equal(nk_g, nk))
    t_g = autotune.time_graph(graph, reps=5)
    del graph
    modes = {}
    for name, mode in (("wave_per_read", QUERY_WAVE_PER_READ), ("work_queue", QUERY_QUEUE)):
        g.set_query_policy(mode, tune.get("chunk", 0) if mode == QUERY_QUEUE else 0,
                           tune.get("waves_per_cu", 0) if mode == QUERY_QUEUE else 0)
        o2 = torch.empty_like(out)
        tm = autotune.time_query_seqs(g, off, ch, o2, nk, reps=5)
        modes[name] = {"reads_per_s": rd.n / tm, "ms": tm * 1e3, "identical": bool(torch.equal(out, o2))}
    g.set_query_policy(0)
    pre = min(args.plain_prefix // 5, rd.n)
    off_p = off[: pre + 1].contiguous()
    g.query_seqs(off_p, ch, plain=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out_p, _ = g.query_seqs(off_p, ch, plain=True)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    same_p = bool(torch.equal(out_p, out[:pre]))
    ceil = roofline.measure(g.index_bytes, n_access=1 << 26, sizes=(4,))["gather"]["4"]["accesses_per_s"]
    rows = full_windows * cfg["R"] * cfg["eta"]
    got = out.cpu().numpy().view(np.uint32)
    g.close()
    # the oracle (literal conjunction over every k-mer, no early exit) on a sample
    nthreads = host_threads()
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, nthreads)
    n_s = min(rd.n, args.oracle_reads)
    so = rd.offsets[: n_s + 1].copy()
    t0 = time.perf_counter()
    want, wn = o.query_seqs(so, rd.chars[: int(so[-1])], nthreads)
    t_o = time.perf_counter() - t0
    o.close()
    same_o = bool(np.array_equal(got[:n_s], want))
    sample_kmers = int(wn.sum())
    log("batched: %.3f ms (%.3g reads/s, %.3g k-mers/s), tile %s, graph replay %.3f ms (identical %s); oracle "
        "%.3g reads/s on %d threads (%d reads, identical %s)"
        % (t_q * 1e3, rd.n / t_q, windows / t_q, tune, t_g * 1e3, same_g, n_s / t_o, nthreads, n_s, same_o))
    return {
        "workload": "batched reads: tiny index (K=64, B=8, R=3, m=2^18, eta=2); %d reads, lognormal "
                    "100-10000 bp (median 1000), 70%% set substrings" % rd.n,
        "reads_per_s": rd.n / t_q, "k_mer_queries_per_s": windows / t_q, "ms": t_q * 1e3, "kmers": windows,
        "tile": {k: tune[k] for k in ("mode", "chunk", "waves_per_cu")},
        "modes": modes,
        "graph_replay": {"reads_per_s": rd.n / t_g, "ms": t_g * 1e3, "identical": same_g},
        "plain_path": {"reads_per_s": pre / t_p, "prefix": pre, "identical": same_p},
        "oracle": {"reads": n_s, "kmers": sample_kmers, "threads": nthreads, "seconds": t_o,
                   "reads_per_s": n_s / t_o, "k_mer_queries_per_s": sample_kmers / t_o, "identical": same_o},
        "roofline": {"kernel": "k_rq_persist" if tune["mode"] != QUERY_WAVE_PER_READ else "k_query_seqs",
                     "bound": "l2-gather", "achieved": rows / t_q, "peak": ceil, "unit": "row gathers/s",
                     "frac": rows / t_q / ceil,
                     "work": "R*eta row gathers per valid window of the reads with a non-empty answer (those "
                             "probe every window in every repetition; reads cut short by the early exit are "
                             "not credited); peak: measured random 4-byte gathers over a buffer of the index's "
                             "size (the 768 KiB index stays in L2)"},
    }


def section_documents(args, steps: int = 3):
    """Word-unigram document index on raw 64-bit keys (Sec. 5.3, the
    Wikipedia sample's shape: K = 17 618 documents, B = 2 000, R = 2,
    m = 200 000, eta = 4) over synthetic Zipf documents: key inserts per
    second, single-word and multi-word queries per second."""
    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo, FLAG_RAW_KEYS
    cfg = synth.INDEX_WIKI
    docs = synth.config_wiki()
    q = synth.word_queries(3006, docs, args.doc_queries)
    ws = synth.word_sets(3007, docs, args.doc_queries, min_words=1, max_words=4)
    g = Rambo(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed=2006, flags=FLAG_RAW_KEYS)
    d = (to_dev(docs.set_ids, np.int32), to_dev(docs.offsets, np.int64), to_dev(docs.keys, np.int64))
    dq = to_dev(q, np.int64)
    dws = (to_dev(ws.offsets, np.int64), to_dev(ws.keys, np.int64))
    out = torch.empty((q.size, g.W), dtype=torch.int32, device="cuda")
    g.insert_kmers(*d)
    g.query_kmers(dq, out=out)
    g.query_termsets(*dws, out=out[: ws.n])
    torch.cuda.synchronize()
    g.set_timing(True)
    g.stage_times()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for e in ev:
        g.clear()
        e[0].record()
        g.insert_kmers(*d)
        e[1].record()
        g.query_kmers(dq, out=out)
        e[2].record()
        g.query_termsets(*dws, out=out[: ws.n])
        e[3].record()
    torch.cuda.synchronize()
    kernels = {k: (v[0] / steps, max(1, v[1] // steps)) for k, v in g.stage_times(calls=True).items()}
    g.set_timing(False)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (documents)")
    t_ins, t_q, t_ws = (float(np.mean([e[i].elapsed_time(e[i + 1]) for e in ev])) for i in range(3))
    n_keys = int(docs.keys.size)
    roofs = insert_rooflines(kernels, n_keys, 0, cfg["R"], cfg["eta"], g.index_bytes, True, "documents",
                             code_input=True)
    qr = query_kmers_roofline(kernels, q.size, cfg["R"], cfg["eta"], g.row_bits, g.W, "documents")
    roofs = sorted(roofs + ([qr] if qr else []), key=lambda r: -r["ms"] * r.get("launches", 1))
    res = {"workload": "word unigrams: K=17618 documents, B=2000, R=2, m=200000, eta=4 (raw 64-bit keys)",
           "keys": n_keys, "queries": int(q.size), "index_bytes": g.index_bytes,
           "insert_ms": t_ins, "keys_inserted_per_s": n_keys / t_ins * 1e3,
           "query_ms": t_q, "word_queries_per_s": q.size / t_q * 1e3,
           "word_sets": {"sets": ws.n, "words": int(ws.keys.size), "query_ms": t_ws, "sets_per_s": ws.n / t_ws * 1e3},
           "kernel_ms": {k: v[0] for k, v in kernels.items()}, "rooflines": roofs}
    log("documents: insert %.2f ms (%.3g keys/s), word queries %.2f ms (%.3g/s), %d word sets %.2f ms (%.3g/s)"
        % (t_ins, res["keys_inserted_per_s"], t_q, res["word_queries_per_s"], ws.n, t_ws,
           res["word_sets"]["sets_per_s"]))
    g.close()
    return res


# ------------------------------------------------------------------ oracle

def host_threads() -> int:
    """Threads for the oracle: the CPU share the process may use (OMP_NUM_THREADS
    when set, else the cores this process may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(sets, rd, kmers_per_read: float, insert_budget: int, query_budget_s: float) -> dict:
    """The oracle, as it stands, on a bounded sample of the headline
    workload: an oracle index of the same shape (K = 100 000, B = 1 000,
    R = 6, m = 2^27: 96 GiB of separate per-cell filters) holding the first
    sets up to `insert_budget` k-mers, then the workload's reads answered one
    after another (literal conjunction over every k-mer, Sec. 3.2.1) for
    about query_budget_s seconds; and the same on one thread."""
    import oracle
    from paper_1910_02611_amd import synth
    cfg = synth.INDEX_LARGE
    nthreads = host_threads()
    lens = np.maximum(sets.lengths().astype(np.int64) - cfg["k"] + 1, 0)
    n_sets = max(1, min(sets.n, int(np.searchsorted(np.cumsum(lens), insert_budget)) + 1))
    sub_off = sets.offsets[: n_sets + 1].copy()
    n_ins = int(lens[:n_sets].sum())
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2005)
    t0 = time.perf_counter()
    o.insert_seqs(sets.set_ids[:n_sets], sub_off, sets.chars[: int(sub_off[-1])], nthreads)
    t_ins = time.perf_counter() - t0
    fill = o.fill_counts().astype(np.float64) / cfg["m"]
    n_r, pos, chunk, kmers = 0, 0, 32 * nthreads, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < query_budget_s:
        a, b = pos, min(pos + chunk, rd.n)
        off = rd.offsets[a:b + 1] - rd.offsets[a]
        _, nk = o.query_seqs(off, rd.chars[int(rd.offsets[a]):int(rd.offsets[b])], nthreads)
        n_r += b - a
        kmers += int(nk.sum())
        pos = b % rd.n
    t_q = time.perf_counter() - t0
    n1, k1, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < 3.0:
        a = n1 % rd.n
        off = rd.offsets[a:a + 2] - rd.offsets[a]
        _, nk = o.query_seqs(off, rd.chars[int(rd.offsets[a]):int(rd.offsets[a + 1])], 1)
        n1 += 1
        k1 += int(nk.sum())
    t1 = time.perf_counter() - t0
    o.close()
    return {
        "value": kmers / t_q, "unit": "k-mer queries/s", "cores": nthreads, "kind": "oracle",
        "value_1_thread": k1 / t1, "reads_per_s": n_r / t_q, "nproc": os.cpu_count(), "cpu": cpu_model(),
        "sample": "the headline workload's reads (150 bp, %.0f 31-mers each), %d of them answered by the oracle in "
                  "%.1f s on %d threads (and %d in %.1f s on one), against an oracle index of the same shape "
                  "(K=100000, B=1000, R=6, m=2^27, eta=2) holding the first %d of the %d sets (%d inserts, %.2f%% "
                  "of the workload's; mean cell fill %.4f, the full index's is higher): the oracle tests all "
                  "B*R*eta filter bits of every k-mer whatever the fill" % (
                      kmers_per_read, n_r, t_q, nthreads, n1, t1, n_sets, sets.n, n_ins,
                      100.0 * n_ins / max(1, int(lens.sum())), float(fill.mean())),
        "inserts_per_s": n_ins / t_ins,
    }


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated subset of %s; the first one run is the headline" % ",".join(SECTIONS))
    ap.add_argument("--large-reads", type=int, default=1_000_000)
    ap.add_argument("--queries", type=int, default=10_000_000, help="k-mer queries of the mid section")
    ap.add_argument("--plain-prefix", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fold", action="store_true")
    ap.add_argument("--no-measured-ceilings", action="store_true")
    ap.add_argument("--doc-queries", type=int, default=1_000_000)
    ap.add_argument("--reads", type=int, default=100_000, help="reads of the batched section")
    ap.add_argument("--oracle-reads", type=int, default=5_000, help="reads of the batched section's oracle sample")
    ap.add_argument("--serve-requests", type=int, default=10_000, help="requests per serving load point")
    ap.add_argument("--serve-loads", default="0.1,0.25,0.4,0.55,0.7,0.85,1.0,1.2")
    ap.add_argument("--serve-slots", type=int, default=4, help="batches in flight at once")
    ap.add_argument("--serve-graphs", action="store_true",
                    help="fixed per-slot buffers and graph replay instead of batches sized from a device pool")
    ap.add_argument("--cpu-insert-budget", type=int, default=60_000_000)
    ap.add_argument("--cpu-query-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune-insert", action="store_true",
                    help="keep the automatic insert tiles instead of autotuning them on the large and mid inserts")
    ap.add_argument("--insert-policy", type=int, default=0,
                    help="rambo_set_insert_policy mode for the large, served and mid indexes (0 = automatic)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run one streaming copy of this size (memory-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this RAMBO build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    sections = [s for s in args.sections.split(",") if s]
    for s in sections:
        if s not in SECTIONS:
            raise SystemExit("unknown section %r" % s)

    import torch
    torch.cuda.set_device(0)
    t_start = time.time()
    res_sec = {}
    large_data = None
    for s in sections:
        t = time.time()
        if s == "large":
            res_sec["large"], sets, rd = section_large(args)
            large_data = (sets, rd)
        elif s == "served":
            if large_data is not None and args.no_cpu_baseline:
                large_data = None
            res_sec["served"] = section_served(args)
        elif s == "mid":
            res_sec["mid"] = section_mid(args)
        elif s == "tiny":
            res_sec["tiny"] = section_tiny(args)
        elif s == "batched":
            res_sec["batched_reads"] = section_batched(args)
        elif s == "documents":
            res_sec["documents"] = section_documents(args)
        log("section %s done in %.1f s (%.1f s so far)" % (s, time.time() - t, time.time() - t_start))
    if args.calib_copy_gib > 0:
        calib_copy(args.calib_copy_gib)

    head_name = "batched_reads" if sections[0] == "batched" else sections[0]
    head = res_sec[head_name]
    if head_name == "large":
        value, roofs = head["k_mer_queries_per_s"], head["rooflines"]
        config = {"workload": head["workload"], "K": head["K"], "B": head["B"], "R": head["R"], "m": head["m"],
                  "eta": head["eta"], "k": head["k"], "inserts": head["inserts"], "reads": head["reads"],
                  "read_kmers": head["read_kmers"]}
    elif head_name == "served":
        value, roofs, config = head["saturated"]["reads_per_s"], head["rooflines"], {"workload": head["workload"]}
    elif head_name == "batched_reads":
        value, roofs, config = head["k_mer_queries_per_s"], [head["roofline"]], {"workload": head["workload"]}
    elif head_name == "documents":
        value, roofs, config = head["word_queries_per_s"], head["rooflines"], {"workload": head["workload"]}
    else:
        value, roofs = head["k_mer_queries_per_s"], head.get("rooflines", [])
        config = {"workload": head["workload"]}
    dominant = [r for r in roofs if r and r["kernel"] != "insert_pipeline"]
    line = {
        "metric": METRIC, "value": value, "unit": "k-mer queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head.get("ms_per_step"), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic", "config": config,
        "inserts_per_s": head.get("inserts_per_s"),
        "roofline": dominant[0] if dominant else None,
        "roofline_other": [r for r in roofs if r and r is not (dominant[0] if dominant else None)],
    }
    if "served" in res_sec:
        sv = res_sec["served"]
        half = min(sv["points"], key=lambda p: abs(p["load"] - 0.55))
        line["latency"] = {"workload": "served (80 GiB index)", "p50_ms": half["p50_ms"], "p99_ms": half["p99_ms"],
                           "load": half["load"], "requests_per_s": half["qps"],
                           "points": [{k: p[k] for k in ("load", "qps", "p50_ms", "p99_ms")} for p in sv["points"]]}
    line.update({k: v for k, v in res_sec.items() if k != head_name})
    line[head_name] = {k: v for k, v in head.items() if k not in ("rooflines",)}
    if not args.no_cpu_baseline and large_data is not None:
        t = time.time()
        sets, rd = large_data
        line["cpu_baseline"] = cpu_baseline(sets, rd, res_sec["large"]["read_kmers"] / max(1, rd.n),
                                            args.cpu_insert_budget, args.cpu_query_seconds)
        log("cpu baseline: %.3g k-mer queries/s on %d threads (%.1f s)"
            % (line["cpu_baseline"]["value"], line["cpu_baseline"]["cores"], time.time() - t))
    log("bench done in %.1f s" % (time.time() - t_start))
    print(json.dumps(line), flush=True)


def calib_copy(gib: float):
    """A streaming copy of known size: the scale of the memory counters."""
    import torch
    from paper_1910_02611_amd.rambo import lib
    n = int(gib * 2**30) // 16 * 16
    buf = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
    assert lib().rambo_roofline_copy(buf.data_ptr(), buf.data_ptr() + n, n,
                                     torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    del buf


if __name__ == "__main__":
    main()
