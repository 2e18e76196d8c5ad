"""Open-loop load driver for the query server (include/rambo_serve.h).

Requests arrive as a Poisson process; a submitter thread hands each one to
the server at its arrival time, and the caller's thread collects the answers.
Latency is arrival -> answer in host memory: the server's own submit ->
result time plus however late the submitter was.  The server, its batching
and every kernel are native.  Two drivers pace the submissions: the native
one (rambo_serve_replay, run_native / sweep_native: no Python between
requests) and a Python one (run_open_loop, which can also interleave insert
requests); this module reports percentiles.

    python -m paper_1910_02611_amd.serve --index tiny --requests 20000
"""
from __future__ import annotations

import argparse
import json
import threading
import time

import numpy as np

from . import rambo, synth


def split_requests(batch: synth.SeqBatch) -> list[tuple[np.ndarray, np.ndarray]]:
    ro = batch.meta["request_offsets"]
    return [synth.request(batch, r) for r in range(len(ro) - 1)]


def run_open_loop(server: rambo.Server, reqs, arrivals: np.ndarray, W: int, inserts=None) -> dict:
    """Submit reqs[i] at arrivals[i] seconds (relative to the start); return
    latencies (ms), throughput and a checksum of the answers.  inserts: an
    optional list of (time, set_ids, offsets, chars) insert requests
    submitted at their times among the queries (streaming updates)."""
    n = len(reqs)
    ids = [None] * n
    lag = np.zeros(n)
    ready = [threading.Event() for _ in range(n)]
    ins = sorted(inserts or [], key=lambda x: x[0])
    ins_ids = []
    t0 = time.perf_counter() + 0.01

    def submitter():
        j = 0
        for i, (off, ch) in enumerate(reqs):
            due = t0 + arrivals[i]
            while j < len(ins) and t0 + ins[j][0] <= due:
                d2 = t0 + ins[j][0]
                now = time.perf_counter()
                if d2 > now:
                    time.sleep(d2 - now)
                ins_ids.append(server.submit_insert(*ins[j][1:]))
                j += 1
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
                now = time.perf_counter()
            ids[i] = server.submit(off, ch)
            lag[i] = max(0.0, now - due)
            ready[i].set()
        for k in range(j, len(ins)):
            ins_ids.append(server.submit_insert(*ins[k][1:]))

    th = threading.Thread(target=submitter)
    th.start()
    lat = np.zeros(n)
    reads = 0
    check = 0
    for i, (off, _) in enumerate(reqs):
        ready[i].wait()
        nr = len(off) - 1
        masks, nk, ms = server.wait(ids[i], nr)
        lat[i] = ms + 1e3 * lag[i]
        reads += nr
        check = (check * 1000003 + int(masks.sum(dtype=np.uint64))) & ((1 << 61) - 1)
    t_end = time.perf_counter()
    th.join()
    span = t_end - t0
    out = dict(requests=n, reads=reads, seconds=span, qps=n / span, reads_per_s=reads / span,
               p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
               mean_ms=float(lat.mean()), max_submit_lag_ms=float(1e3 * lag.max()), checksum=check)
    if ins:
        il = np.array([server.wait_insert(r) for r in ins_ids])
        out.update(inserts=len(ins), insert_bases=int(sum(int(x[2][-1]) for x in ins)),
                   insert_p50_ms=float(np.percentile(il, 50)), insert_p99_ms=float(np.percentile(il, 99)))
    return out


def run_native(server: rambo.Server, batch: synth.SeqBatch, arrivals: np.ndarray) -> dict:
    """The same measurement with the native driver (rambo_serve_replay): the
    requests of a served_requests batch submitted at their arrival times
    from a native thread, no Python between the requests."""
    ro = batch.meta["request_offsets"]
    server.worker_stats(reset=True)
    thr0 = cpu_throttling()
    t0 = time.perf_counter()
    lat, check, qms = server.replay(ro, batch.offsets, batch.chars, arrivals, with_queue=True)
    span = time.perf_counter() - t0
    thr1 = cpu_throttling()
    n = ro.size - 1
    reads = int(ro[-1] - ro[0])
    out = dict(requests=n, reads=reads, seconds=span, qps=n / span, reads_per_s=reads / span,
               p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
               mean_ms=float(lat.mean()), checksum=int(check),
               queue_p50_ms=float(np.percentile(qms, 50)), queue_p99_ms=float(np.percentile(qms, 99)),
               service_p99_ms=float(np.percentile(lat - qms, 99)))
    if thr0 is not None and thr1 is not None:
        out["cpu_throttled_periods"] = thr1[0] - thr0[0]
        out["cpu_throttled_ms"] = (thr1[1] - thr0[1]) / 1e3
    out.update({"worker_" + k: v for k, v in server.worker_stats().items()})
    return out


def cpu_throttling():
    """(periods throttled, microseconds throttled) of this process's cgroup
    CPU quota so far (cpu.stat of cgroup v2, else v1), or None where
    neither is readable."""
    for path, key, scale in (("/sys/fs/cgroup/cpu.stat", "throttled_usec", 1),
                             ("/sys/fs/cgroup/cpu/cpu.stat", "throttled_time", 1000),
                             ("/sys/fs/cgroup/cpu,cpuacct/cpu.stat", "throttled_time", 1000)):
        try:
            with open(path) as f:
                kv = dict(line.split() for line in f if line.strip())
            return int(kv.get("nr_throttled", 0)), int(kv.get(key, 0)) // scale
        except (OSError, ValueError):
            continue
    return None


def sweep_native(server: rambo.Server, batch: synth.SeqBatch, fractions, seed: int = 5004) -> dict:
    """Saturated rate (every request at time 0), then Poisson load at the
    given fractions of it, with the native driver."""
    n = batch.meta["request_offsets"].size - 1
    sat = run_native(server, batch, np.zeros(n))
    points = []
    for j, f in enumerate(fractions):
        rate = f * sat["qps"]
        r = run_native(server, batch, synth.poisson_arrivals(seed + j, n, rate))
        r["offered_qps"] = rate
        r["load"] = f
        points.append(r)
    return dict(saturated=sat, points=points)


def saturated(server: rambo.Server, reqs, W: int) -> dict:
    """Every request queued at once: the server's peak request rate."""
    return run_open_loop(server, reqs, np.zeros(len(reqs)), W)


def sweep(server: rambo.Server, reqs, W: int, fractions, seed: int = 5004, per_point: int | None = None) -> dict:
    """Saturated throughput, then Poisson load at the given fractions of it."""
    sat = saturated(server, reqs, W)
    points = []
    for j, f in enumerate(fractions):
        sub = reqs if per_point is None else reqs[:per_point]
        rate = f * sat["qps"]
        arr = synth.poisson_arrivals(seed + j, len(sub), rate)
        r = run_open_loop(server, sub, arr, W)
        r["offered_qps"] = rate
        r["load"] = f
        points.append(r)
    return dict(saturated=sat, points=points)


def insert_stream(seed: int, sets: synth.SeqBatch, n_inserts: int, period_s: float, seqs_per_insert: int,
                  seq_len: int) -> list:
    """n_inserts insert requests, one every period_s seconds, each of
    seqs_per_insert pieces of seq_len bases cut from random set genomes and
    added to random sets (new terms for those sets)."""
    rng = synth.rng_for(seed)
    lens = sets.lengths().astype(np.int64)
    out = []
    for j in range(n_inserts):
        src = rng.integers(0, sets.n, size=seqs_per_insert)
        parts = []
        for s in src:
            L = min(seq_len, int(lens[s]))
            a = int(sets.offsets[s]) + int(rng.integers(0, int(lens[s]) - L + 1))
            parts.append(sets.chars[a:a + L])
        off = np.zeros(seqs_per_insert + 1, np.uint64)
        np.cumsum([p.size for p in parts], out=off[1:])
        ids = rng.integers(0, int(sets.set_ids.max()) + 1, size=seqs_per_insert).astype(np.uint32)
        out.append(((j + 1) * period_s, ids, off, np.concatenate(parts)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--index", choices=["tiny", "mid", "served"], default="tiny")
    ap.add_argument("--requests", type=int, default=10_000)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--graphs", action="store_true")
    ap.add_argument("--loads", default="0.1,0.25,0.4,0.55,0.7,0.85,1.0,1.2")
    args = ap.parse_args()
    import torch

    sets = {"tiny": synth.config_tiny, "mid": synth.config_mid, "served": synth.config_served}[args.index]()
    params = {"tiny": synth.INDEX_TINY, "mid": synth.INDEX_MID, "served": synth.INDEX_SERVED}[args.index]
    idx = rambo.Rambo(**params, seed={"tiny": 2001, "mid": 2002, "served": 2004}[args.index])
    dev = torch.device("cuda")
    idx.insert_seqs(torch.from_numpy(sets.set_ids.view(np.int32)).to(dev),
                    torch.from_numpy(sets.offsets.view(np.int64)).to(dev),
                    torch.from_numpy(sets.chars).to(dev))
    torch.cuda.synchronize()
    batch = synth.served_requests(4004, sets, args.requests)
    del sets
    with rambo.Server(idx, max_slots=args.slots, use_graphs=args.graphs) as srv:
        res = sweep_native(srv, batch, [float(x) for x in args.loads.split(",")])
        res["server"] = srv.stats()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
