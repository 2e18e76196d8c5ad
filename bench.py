#!/usr/bin/env python3
"""RAMBO on one MI355X: bulk insertion and batched k-mer queries.

Workload (synthetic, seeded): K = 1 000 genome sets, lognormal lengths
(median 200 kbp, 20 kbp - 2 Mbp) cut from 50 random 2 Mbp ancestors with 1%
substitutions (~2.7e8 31-mers); index B = 50, R = 4, m = 2^28 bits per cell,
eta = 2 (8 GiB bit-sliced); 1e7 single 31-mer queries, half drawn from the
inserted genomes, half uniform random.

One step = zero the index + insert every set (partitioned insert, or
k_insert_seqs for small inserts) + answer every query (k_query_kmers).
Inputs are resident in device memory before timing.  `value` is k-mer
queries per second of the query phase; inserts per second of the insert
phase are reported beside it.  Phase times come from HIP events recorded on
the stream the kernels run on.

Further sections of the same JSON line: the one-launch-per-query comparator
(`plain_path`), the query server on the mid index with and without streaming
inserts (`serving`, `latency`), batched reads on the small index
(`batched_reads`), folding the mid index over (`fold`), the word-unigram
document index on raw 64-bit keys (`documents`) and the oracle on the host
(`cpu_baseline`).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
SECTOR = 64             # bytes moved per random access at HBM (one sector)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(n_queries: int):
    from paper_1910_02611_amd import synth
    t = time.time()
    sets = synth.config_mid()
    q = synth.kmer_queries(3002, sets, n_queries, 31)
    log("workload: %d sets, %d bases, %d queries (%.1f s)" % (sets.n, sets.chars.size, q.n, time.time() - t))
    return sets, q


def to_dev(a, view):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(view)).to("cuda")


def time_steps(g, dsets, codes, out, steps: int, warmup: int):
    import torch
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]

    def one_step(e=None):
        if e: e[0].record(stream)
        g.clear()
        if e: e[1].record(stream)
        g.insert_seqs(*dsets)
        if e: e[2].record(stream)
        g.query_kmers(codes, out=out)
        if e: e[3].record(stream)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    g.stage_times()        # drop anything recorded so far
    g.set_timing(True)     # per-kernel HIP events on the same stream, inside the library
    t0 = time.perf_counter()
    for s in range(steps):
        one_step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.set_timing(False)
    kernels = {k: v / steps for k, v in g.stage_times().items()}
    clear = np.mean([e[0].elapsed_time(e[1]) for e in ev])
    ins = np.mean([e[1].elapsed_time(e[2]) for e in ev])
    qry = np.mean([e[2].elapsed_time(e[3]) for e in ev])
    return wall, clear, ins, qry, kernels


# Integer work of the binning kernel's algorithm, in 32-bit VALU operations
# (64-bit shift 1, 64-bit xor/add 2, 64x64 multiply 5): extracting one
# canonical window from the packed streams and mixing it once (two
# xorshift-multiply rounds and a final xorshift: 19), and per bit target the
# multiply-shift position (5 + 1), the bit address (4) and its bucket split
# (2).
ALU_OPS_PER_WINDOW = 30 + 19
ALU_OPS_PER_TARGET = 12
# a raw 64-bit key is only mixed (19) before its bit targets
ALU_OPS_PER_KEY = 19
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # CUs x SIMDs x lanes x clock: 39.3 T int32 ops/s
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
TRAFFIC_JSON = os.path.join(PROFILES, "traffic_mid.json")
TRAFFIC_DOCS_JSON = os.path.join(PROFILES, "traffic_documents.json")


def measured_traffic(names: dict, path: str = TRAFFIC_JSON) -> dict:
    """HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE) from the
    committed rocprofv3 summary of one workload, for stage name -> kernel
    name as profiled; empty when the summary is missing or the kernel sources
    changed since."""
    from paper_1910_02611_amd.profsum import load_traffic
    t = load_traffic(path)
    if t is None:
        return {}
    return {stage: t["kernels"][k]["bytes"] for stage, k in names.items() if k in t["kernels"]}


def kernel_rooflines(kernels, n_ins, n_queries, R, eta, S, W, index_bytes, fresh=True, traffic_json=TRAFFIC_JSON,
                     term_sets=0, set_terms=0):
    """Roofline entry of each timed kernel: algorithmic work per launch over
    its measured duration.  fresh: the insert went into an all-zero index,
    so stage C writes the index without reading it.  traffic_json: the
    profiled HBM bytes of this workload's launches."""
    RE = R * eta
    SW = max(1, S // 32)
    targets = n_ins * RE
    work = {
        "k_bin_windows": ("alu", n_ins * (ALU_OPS_PER_WINDOW + RE * ALU_OPS_PER_TARGET), "TOP/s",
                          "int32 VALU ops: %d per window + %d per target" % (ALU_OPS_PER_WINDOW, ALU_OPS_PER_TARGET)),
        "k_bin_codes": ("alu", n_ins * (ALU_OPS_PER_KEY + RE * ALU_OPS_PER_TARGET), "TOP/s",
                        "int32 VALU ops: %d per raw key + %d per target" % (ALU_OPS_PER_KEY, ALU_OPS_PER_TARGET)),
        "k_bin_regions": ("hbm", targets * 8, "GB/s", "4 B read + 4 B written per bit target"),
        "k_apply_regions": ("hbm", targets * 4 + (1 if fresh else 2) * index_bytes, "GB/s",
                            "4 B read per bit target + index written once (and read once unless the index "
                            "was all zero)"),
        "k_insert_seqs": ("hbm", n_ins * RE * 2 * SECTOR, "GB/s", "one 64-B sector read-modify-write per target"),
        "k_insert_kmers": ("hbm", n_ins * RE * 2 * SECTOR, "GB/s", "one 64-B sector read-modify-write per target"),
        "k_query_kmers": ("hbm", n_queries * (RE * max(SECTOR, S // 8) + 4 * W + 8), "GB/s",
                          "R*eta row sectors + K-bit answer + code per query"),
        "k_query_termsets": ("hbm", set_terms * (RE * max(SECTOR, S // 8) + 8) + term_sets * (4 * W + 8), "GB/s",
                             "R*eta row sectors + code per term (no early exit subtracted), K-bit answer + "
                             "offset per set"),
    }
    launch_bytes = measured_traffic({"k_bin_windows": "k_bin_windows_hold<%d, %d>" % (R, eta),
                                     "k_bin_codes": "k_bin_codes_hold<%d, %d>" % (R, eta),
                                     "k_insert_kmers": "k_insert_kmers",
                                     "k_bin_regions": "k_bin_regions", "k_apply_regions": "k_apply_regions",
                                     "k_insert_seqs": "k_insert_seqs<%d, %d>" % (R, eta),
                                     "k_query_kmers": "k_query_kmers<%d, %d, %d>" % (SW, R, eta),
                                     "k_query_termsets": "k_query_termsets<%d, %d, %d>" % (SW, R, eta)},
                                    traffic_json)
    out = []
    for name, ms in kernels.items():
        if name not in work:
            continue
        bound, amount, unit, what = work[name]
        sec = ms / 1e3
        if bound == "alu":
            achieved, peak = amount / sec / 1e12, VALU_PEAK_TOPS
        else:
            achieved, peak = amount / sec / 1e9, HBM_PEAK_GBS
        out.append({"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                    "frac": achieved / peak, "traffic": launch_bytes.get(name), "ms": ms,
                    "work_per_launch": amount, "work": what})
    out.sort(key=lambda r: -r["ms"])
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
    same = bool(torch.equal(got, out_batched[:n_prefix]))
    return n_prefix / dt, same


def cpu_baseline(sets, q, cfg, query_budget_s: float = 12.0):
    """The oracle, as it stands, on a bounded sample: the index built from the
    first sets (until ~5e7 k-mers), then queries of the same stream, repeated
    for about query_budget_s seconds."""
    import oracle
    nthreads = min(os.cpu_count() or 1, 16)
    lens = sets.lengths().astype(np.int64)
    n_sets = int(np.searchsorted(np.cumsum(lens), 50_000_000)) + 1
    n_sets = max(1, min(n_sets, sets.n))
    sub_off = sets.offsets[: n_sets + 1].copy()
    sub_chars = sets.chars[: int(sub_off[-1])]
    n_ins = int(np.sum(np.maximum(lens[:n_sets] - cfg["k"] + 1, 0)))
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2002)
    t0 = time.perf_counter()
    o.insert_seqs(sets.set_ids[:n_sets], sub_off, sub_chars, nthreads)
    t_ins = time.perf_counter() - t0
    nq = min(q.n, 2_000_000)
    k = cfg["k"]
    codes = oracle.extract(q.offsets[: nq + 1], q.chars[: nq * k], k)[q.offsets[:nq].astype(np.int64)]
    n_q, pos, chunk = 0, 0, 200_000
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < query_budget_s:
        o.query_kmers(codes[pos:pos + chunk], nthreads)
        n_q += min(chunk, nq - pos)
        pos = (pos + chunk) % nq
    t_q = time.perf_counter() - t0
    # one host thread (the setting of the paper's own timings), briefly
    n1, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 2.0:
        o.query_kmers(codes[n1 % nq:n1 % nq + 20_000], 1)
        n1 += min(20_000, nq - n1 % nq)
    t1 = time.perf_counter() - t0
    o.close()
    return {
        "value": n_q / t_q, "unit": "k-mer queries/s", "cores": nthreads, "kind": "oracle",
        "value_1_thread": n1 / t1,
        "sample": "%d k-mer queries (the first %d of the same stream, cycled) against the oracle index of "
                  "the first %d of %d sets; oracle insert of those sets: %d inserts in %.1f s (%.3g inserts/s)"
                  % (n_q, nq, n_sets, sets.n, n_ins, t_ins, n_ins / t_ins),
        "inserts_per_s": n_ins / t_ins,
    }


def batched_reads(n_reads: int, plain_prefix: int = 2000):
    """Batched sequence queries (Sec. 3.2.1) on the tiny index: 64 sets, B=8,
    R=3, m=2^18; reads of lognormal length (median 1 000, 100-10 000 bp), 70%
    substrings of a set genome.  One persistent work-queue launch with the
    autotuned tile, against one wave per read and one launch per read."""
    import torch
    from paper_1910_02611_amd import autotune, synth
    from paper_1910_02611_amd.rambo import Rambo, QUERY_WAVE_PER_READ

    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    g = Rambo(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed=2001)
    g.insert_seqs(to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    t = time.time()
    rd = synth.config_batched_reads(sets, n_reads)
    log("batched reads: %d reads, %d bases (%.1f s)" % (rd.n, rd.chars.size, time.time() - t))
    off, ch = to_dev(rd.offsets, np.int64), to_dev(rd.chars, np.uint8)
    tune = autotune.tune_query_seqs(g, off, ch, tag="batched-reads", use_cache=False)
    out = torch.empty((rd.n, g.W), dtype=torch.int32, device="cuda")
    nk = torch.empty(rd.n, dtype=torch.int32, device="cuda")
    t_q = autotune.time_query_seqs(g, off, ch, out, nk, reps=5)
    windows = int(nk.to(torch.int64).sum())
    # reads with a non-empty answer probe every window in every repetition
    full_windows = int(nk.to(torch.int64)[out.ne(0).any(dim=1)].sum())
    # the same batch as one captured graph, replayed with eager calls in
    # between; every replay must give the eager answers
    out_g = torch.empty_like(out)
    nk_g = torch.empty_like(nk)
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
    g.set_query_policy(QUERY_WAVE_PER_READ)
    out_w = torch.empty_like(out)
    t_w = autotune.time_query_seqs(g, off, ch, out_w, nk, reps=5)
    same_w = bool(torch.equal(out, out_w))
    # one launch per read on a prefix
    pre = min(plain_prefix, rd.n)
    off_p = off[: pre + 1].contiguous()
    g.query_seqs(off_p, ch, plain=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out_p, _ = g.query_seqs(off_p, ch, plain=True)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    same_p = bool(torch.equal(out_p, out[:pre]))
    # the index (768 KiB) stays in L2: the ceiling is the measured rate of
    # random 4-byte gathers over a buffer of the index's size
    from paper_1910_02611_amd import roofline
    ceil = roofline.measure(g.index_bytes, n_access=1 << 26, sizes=(4,))["gather"]["4"]["accesses_per_s"]
    rows = full_windows * cfg["R"] * cfg["eta"]
    g.close()
    log("batched reads: tuned %.3f ms (%.3g reads/s, %.3g k-mers/s), graph replay %.3f ms (identical %s), "
        "wave-per-read %.3f ms, plain %.3g reads/s"
        % (t_q * 1e3, rd.n / t_q, windows / t_q, t_g * 1e3, same_g, t_w * 1e3, pre / t_p))
    return {
        "workload": "batched reads: tiny index (K=64, B=8, R=3, m=2^18, eta=2); %d reads, lognormal "
                    "100-10000 bp (median 1000), 70%% set substrings" % rd.n,
        "reads_per_s": rd.n / t_q, "k_mer_queries_per_s": windows / t_q, "ms": t_q * 1e3, "kmers": windows,
        "tile": {k: tune[k] for k in ("mode", "chunk", "waves_per_cu")},
        "wave_per_read": {"reads_per_s": rd.n / t_w, "ms": t_w * 1e3, "identical": same_w},
        "graph_replay": {"reads_per_s": rd.n / t_g, "ms": t_g * 1e3, "identical": same_g},
        "plain_path": {"reads_per_s": pre / t_p, "prefix": pre, "identical": same_p},
        "roofline": {"kernel": "k_rq_persist" if tune["mode"] != QUERY_WAVE_PER_READ else "k_query_seqs",
                     "bound": "l2-gather", "achieved": rows / t_q, "peak": ceil, "unit": "row gathers/s",
                     "frac": rows / t_q / ceil,
                     "work": "R*eta row gathers per valid window of the reads with a non-empty answer (those "
                             "probe every window in every repetition; reads cut short by the early exit are "
                             "not credited); peak: measured random 4-byte gathers over a buffer of the index's "
                             "size"},
    }


def serving(g, sets, n_requests: int, loads, slots: int = 4):
    """The query server on the resident index: requests of U{1..64} reads,
    lengths log-uniform in [150, 5000] bp, 70% set substrings; saturated rate
    (all requests queued at once), then Poisson arrivals at fractions of it.
    Latency = arrival -> answer in host memory."""
    from paper_1910_02611_amd import serve, synth
    from paper_1910_02611_amd.rambo import Server

    t = time.time()
    batch = synth.served_requests(4004, sets, n_requests)
    reqs = serve.split_requests(batch)
    log("serving: %d requests, %d reads (%.1f s)" % (len(reqs), sum(len(o) - 1 for o, _ in reqs), time.time() - t))
    with Server(g, max_slots=slots, use_graphs=True) as srv:
        serve.saturated(srv, reqs[: min(200, len(reqs))], g.W)   # warm-up
        # submissions paced by a native thread (no Python between requests)
        res = serve.sweep_native(srv, batch, loads)
        # streaming inserts among the queries (every 20 ms, 32 pieces of 5
        # kbp added to random sets) against the same arrivals without them;
        # the Python driver paces both, at a quarter of the saturated rate
        rate = 0.25 * res["saturated"]["qps"]
        arr = synth.poisson_arrivals(5100, len(reqs), rate)
        ins = serve.insert_stream(5101, sets, max(1, int(arr[-1] / 0.02)), 0.02, 32, 5000)
        plain = serve.run_open_loop(srv, reqs, arr, g.W)
        mixed = serve.run_open_loop(srv, reqs, arr, g.W, inserts=ins)
        res["server"] = srv.stats()
    sat = res["saturated"]
    log("serving at load 0.25 (Python driver): query p50 %.3f ms p99 %.3f ms; with %d inserts of %d bases: "
        "query p50 %.3f ms p99 %.3f ms, insert p50 %.3f ms p99 %.3f ms"
        % (plain["p50_ms"], plain["p99_ms"], mixed["inserts"], mixed["insert_bases"] // mixed["inserts"],
           mixed["p50_ms"], mixed["p99_ms"], mixed["insert_p50_ms"], mixed["insert_p99_ms"]))
    log("serving: saturated %.4g requests/s (%.4g reads/s), p50 %.3f ms p99 %.3f ms"
        % (sat["qps"], sat["reads_per_s"], sat["p50_ms"], sat["p99_ms"]))
    for p in res["points"]:
        log("  load %.2f: offered %.4g/s achieved %.4g/s  p50 %.3f ms  p99 %.3f ms"
            % (p["load"], p["offered_qps"], p["qps"], p["p50_ms"], p["p99_ms"]))
    keep = ("load", "offered_qps", "qps", "reads_per_s", "p50_ms", "p99_ms", "mean_ms")
    return {
        "workload": "served requests on the resident index: U{1..64} reads of log-uniform 150-5000 bp, "
                    "70%% set substrings; %d requests per point, %d slots, graph replay; native open-loop "
                    "driver (with_inserts: the Python driver)" % (len(reqs), slots),
        "saturated": {k: sat[k] for k in ("qps", "reads_per_s", "p50_ms", "p99_ms")},
        "points": [{k: p[k] for k in keep} for p in res["points"]],
        "with_inserts": dict({k: mixed[k] for k in ("qps", "p50_ms", "p99_ms", "inserts", "insert_bases",
                                                    "insert_p50_ms", "insert_p99_ms")},
                             load=0.25, without_inserts={k: plain[k] for k in ("qps", "p50_ms", "p99_ms")}),
        "server": res["server"],
    }


def documents(n_queries: int, steps: int = 3):
    """Word-unigram document index on raw 64-bit keys (Sec. 5.3, the
    Wikipedia sample's shape: K = 17 618 documents, B = 2 000, R = 2,
    m = 200 000, eta = 4) over synthetic Zipf documents (about 1.7e7
    distinct document-word pairs): key inserts per second and single-word
    queries per second, each phase timed with HIP events, with the roofline
    of its kernel."""
    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo, FLAG_RAW_KEYS
    cfg = synth.INDEX_WIKI
    t = time.time()
    docs = synth.config_wiki()
    q = synth.word_queries(3006, docs, n_queries)
    ws = synth.word_sets(3007, docs, n_queries, min_words=1, max_words=4)
    log("documents: %d docs, %d keys, %d queries (%.1f s to generate)" % (docs.n, docs.keys.size, q.size,
                                                                         time.time() - t))
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
    kernels = {k: v / steps for k, v in g.stage_times().items()}
    g.set_timing(False)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set (documents)")
    t_ins = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    t_q = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    t_ws = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
    n_keys, RE, S, W = int(docs.keys.size), cfg["R"] * cfg["eta"], g.row_bits, g.W
    # every timed insert follows a clear: stage C writes without reading back
    roofs = kernel_rooflines(kernels, n_keys, q.size, cfg["R"], cfg["eta"], S, W, g.index_bytes, fresh=True,
                             traffic_json=TRAFFIC_DOCS_JSON, term_sets=ws.n, set_terms=int(ws.keys.size))
    ins_ms = kernels.get("k_insert_kmers")
    if ins_ms:
        # the direct insert (chosen for small batches): the 100 MB index sits
        # largely in the 256 MB last-level cache, so its ceiling is the
        # measured rate of random 32-bit atomicOr over a buffer of the index's
        # size
        from paper_1910_02611_amd import roofline
        atomic_peak = roofline.measure(g.index_bytes, n_access=1 << 26, sizes=())["atomic_or"]["accesses_per_s"]
        a = n_keys * RE / (ins_ms / 1e3)
        roofs.append({"kernel": "k_insert_kmers", "bound": "atomic", "achieved": a, "peak": atomic_peak,
                      "unit": "atomicOr/s", "frac": a / atomic_peak, "ms": ins_ms, "work_per_launch": n_keys * RE,
                      "work": "R*eta random 32-bit atomicOr per key; peak: measured random atomicOr over a "
                              "buffer of the index's size"})
    res = {"workload": "word unigrams: K=17618 documents, B=2000, R=2, m=200000, eta=4 (raw 64-bit keys)",
           "keys": n_keys, "queries": int(q.size), "index_bytes": g.index_bytes,
           "insert_ms": t_ins, "keys_inserted_per_s": n_keys / t_ins * 1e3,
           "query_ms": t_q, "word_queries_per_s": q.size / t_q * 1e3,
           "word_sets": {"sets": ws.n, "words": int(ws.keys.size), "query_ms": t_ws,
                         "sets_per_s": ws.n / t_ws * 1e3,
                         "what": "1-4 words per query, half of them from one document, answered by "
                                 "rambo_query_termsets (the documents holding every word)"},
           "kernel_ms": kernels, "rooflines": roofs}
    log("documents: insert %.2f ms (%.3g keys/s), query %.2f ms (%.3g queries/s), %d word sets %.2f ms "
        "(%.3g sets/s)" % (t_ins, res["keys_inserted_per_s"], t_q, res["word_queries_per_s"], ws.n, t_ws,
                           res["word_sets"]["sets_per_s"]))
    for r in roofs:
        log("  %-16s %8.3f ms  %-6s %.3g %s (%.1f%%)" % (r["kernel"], r["ms"], r["bound"], r["achieved"], r["unit"],
                                                      100 * r["frac"]))
    g.close()
    return res


def measured_ceilings(index_bytes: int, S: int, RE: int, q_per_s: float, ins_per_s: float) -> dict:
    """Both phases against ceilings measured on this GPU over a buffer as large
    as the index (so TLB and last-level-cache effects are included): k-mer
    queries against random gathers of one row (S/8 bytes, at least 4), each
    query credited with all R*eta rows (the early exit is not subtracted);
    inserts against random 32-bit atomicOr, each insert needing R*eta bit
    sets - the rate a one-atomic-per-target insert could reach."""
    from paper_1910_02611_amd import roofline
    G = max(4, S // 8)
    m = roofline.measure(index_bytes, n_access=1 << 27, sizes=(G,))
    gathers = m["gather"][str(G)]["accesses_per_s"]
    atomics = m["atomic_or"]["accesses_per_s"]
    log("measured ceilings over %.1f GiB: random %d-byte gathers %.3g/s, random atomicOr %.3g/s"
        % (index_bytes / 2**30, G, gathers, atomics))
    return {"buffer_bytes": index_bytes,
            "query": {"achieved": q_per_s * RE, "ceiling": gathers, "unit": "row gathers/s",
                      "frac": q_per_s * RE / gathers, "row_bytes": G},
            "insert": {"achieved": ins_per_s * RE, "ceiling": atomics, "unit": "bit targets/s",
                       "frac": ins_per_s * RE / atomics}}


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
    achieved = moved / (ms / 1e3) / 1e9
    kname = {32: "k_fold_narrow<1>", 64: "k_fold_narrow<2>"}.get(g.row_bits, "k_fold")
    log("fold B %d -> %d: k_fold %.3f ms (%.0f GB/s, %.1f%% of HBM peak), call %.1f ms"
        % (B, g.B, ms, achieved, 100 * achieved / HBM_PEAK_GBS, wall * 1e3))
    return {"B_from": B, "B_to": g.B, "index_bytes_from": old_bytes, "index_bytes_to": g.index_bytes,
            "call_ms": wall * 1e3,
            "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic({"k_fold": kname}).get("k_fold"), "ms": ms,
                         "work_per_launch": moved, "work": "old index read once + folded index written once"}}


def calib_copy(gib: float):
    """A streaming copy of known size (none for 0): the scale of the memory
    counters."""
    if gib <= 0:
        return
    import torch
    from paper_1910_02611_amd.rambo import lib
    n = int(gib * 2**30) // 16 * 16
    buf = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
    assert lib().rambo_roofline_copy(buf.data_ptr(), buf.data_ptr() + n, n,
                                     torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    del buf


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=10_000_000)
    ap.add_argument("--plain-prefix", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fold", action="store_true", help="skip folding the index over at the end")
    ap.add_argument("--no-measured-ceilings", action="store_true",
                    help="skip measuring the random-gather and random-atomic ceilings over an index-sized buffer")
    ap.add_argument("--doc-queries", type=int, default=1_000_000,
                    help="word queries of the document-index section (0 = skip)")
    ap.add_argument("--reads", type=int, default=100_000, help="batched-read section size (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=3000, help="requests per serving load point (0 = skip)")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.8,1.0")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run one streaming copy of this size (memory-counter calibration)")
    ap.add_argument("--documents-only", action="store_true",
                    help="run only the document-index section (its own profile), printing its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: RAMBO's hot path here has no multi-GPU part "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_02611_amd import synth
    from paper_1910_02611_amd.rambo import Rambo

    torch.cuda.set_device(0)
    if args.documents_only:
        res = {"documents": documents(args.doc_queries, steps=args.steps)}
        calib_copy(args.calib_copy_gib)
        print(json.dumps(res), flush=True)
        return
    cfg = synth.INDEX_MID
    sets, q = build_workload(args.queries)
    g = Rambo(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], seed=2002)
    dsets = (to_dev(sets.set_ids, np.int32), to_dev(sets.offsets, np.int64), to_dev(sets.chars, np.uint8))
    qoff = to_dev(q.offsets, np.int64)
    qchars = to_dev(q.chars, np.uint8)
    codes = g.extract_kmers(qoff, qchars)[qoff[:-1]].contiguous()
    del qchars
    out = torch.empty((q.n, g.W), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    log("index: %.2f GiB, row %d bits, %d answer words" % (g.index_bytes / 2**30, g.row_bits, g.W))

    wall, t_clear, t_ins, t_q, kernels = time_steps(g, dsets, codes, out, args.steps, args.warmup)
    if g.sync_status() != 0:
        raise SystemExit("device error flag set")
    n_ins = int(np.sum(np.maximum(sets.lengths().astype(np.int64) - cfg["k"] + 1, 0)))
    ins_per_s = n_ins / (t_ins / 1e3)
    q_per_s = q.n / (t_q / 1e3)
    ms_per_step = wall / args.steps * 1e3
    log("step %.2f ms: clear %.2f, insert %.2f (%.3g inserts/s), query %.2f (%.3g queries/s)"
        % (ms_per_step, t_clear, t_ins, ins_per_s, t_q, q_per_s))

    R, eta, S, W = cfg["R"], cfg["eta"], g.row_bits, g.W
    roofs = kernel_rooflines(kernels, n_ins, q.n, R, eta, S, W, g.index_bytes)
    for r in roofs:
        log("  %-16s %8.3f ms  %-3s %.3g %s (%.1f%% of %.4g)" % (r["kernel"], r["ms"], r["bound"], r["achieved"],
                                                               r["unit"], 100 * r["frac"], r["peak"]))

    measured = None
    if not args.no_measured_ceilings:
        measured = measured_ceilings(g.index_bytes, S, R * eta, q_per_s, ins_per_s)
    calib_copy(args.calib_copy_gib)
    plain_rate, plain_same = None, None
    if args.plain_prefix > 0:
        plain_rate, plain_same = plain_path(g, codes, out, min(args.plain_prefix, q.n))
        log("plain one-launch-per-query path: %.3g queries/s on %d, identical=%s"
            % (plain_rate, args.plain_prefix, plain_same))

    res = {
        "metric": "k-mer queries/s and inserts/s on 1 GPU (% of random-HBM roofline); p50/p99 latency",
        "value": q_per_s, "unit": "k-mer queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "mid: K=1000 genome sets (~2.7e8 31-mers), B=50, R=4, m=2^28, eta=2; "
                               "1e7 single 31-mer queries (50% present)",
                   "K": cfg["K"], "B": cfg["B"], "R": cfg["R"], "m": cfg["m"], "eta": cfg["eta"],
                   "k": cfg["k"], "inserts": n_ins, "queries": q.n},
        "inserts_per_s": ins_per_s,
        "phase_ms": {"clear": t_clear, "insert": t_ins, "query": t_q},
        "kernel_ms": kernels,
        "roofline": roofs[0], "roofline_other": roofs[1:], "measured_ceilings": measured,
        "plain_path": {"k_mer_queries_per_s": plain_rate, "prefix": args.plain_prefix,
                       "identical": plain_same, "speedup_batched": q_per_s / plain_rate if plain_rate else None},
    }
    if args.serve_requests > 0:
        res["serving"] = serving(g, sets, args.serve_requests, [float(x) for x in args.serve_loads.split(",")])
        half = min(res["serving"]["points"], key=lambda p: abs(p["load"] - 0.5))
        res["latency"] = {"p50_ms": half["p50_ms"], "p99_ms": half["p99_ms"], "load": half["load"],
                          "requests_per_s": half["qps"]}
    if not args.no_fold:
        res["fold"] = fold_timing(g)
    g.close()
    del out, codes, dsets
    torch.cuda.empty_cache()
    if args.reads > 0:
        res["batched_reads"] = batched_reads(args.reads)
    if args.doc_queries > 0:
        res["documents"] = documents(args.doc_queries)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        t = time.time()
        res["cpu_baseline"] = cpu_baseline(sets, q, cfg)
        log("cpu baseline: %.3g queries/s (%.1f s)" % (res["cpu_baseline"]["value"], time.time() - t))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
