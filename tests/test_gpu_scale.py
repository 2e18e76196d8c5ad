"""Parity at the full size of the served and large workloads (10 000 sets,
B = 200, R = 5, m = 2^29: an 80 GiB index; 100 000 sets, B = 1 000, R = 6,
m = 2^27: a 96 GiB index), inserted in the launch configuration bench.py
times (rambo_insert_seqs, automatic policy: the partitioned insert in scratch
batches).  The oracle cannot hold these indexes, so it checks outputs it can
compute one by one:
  - for a sample of sets s: the R cells (r, phi_r(s)) that hold s, built by
    the oracle from the sets in them alone (Alg. 1 for one cell), compared
    bit for bit with those columns of the device index (every row);
  - for the same sets, the membership bit of every sampled read and k-mer
    query (Sec. 3.2.1, Alg. 2: s is in an answer iff all its R cells pass
    every valid window), compared with the device masks and ID lists;
and, on many more reads, the device answers contain every read's source set
(no false negatives).  With RAMBO_SCALE_ROWS=1 a slower check also runs: the
oracle passes over every window of every set once and compares every row
p = 0 mod D of every repetition, bit for bit, and the full answers of a
sample of reads (D = 256, 64 with RAMBO_SCALE_FULL=1; 3 to 7 minutes of host
time).  RAMBO_SCALE (comma-separated: served, large, mini) chooses the
workloads; both full-size ones run by default.  Progress lines go to
gpurun_out/scale_progress.log as the long host steps advance."""
import json
import os
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import serve, synth
from gpu_util import dev, host_u32

SCALE = [s for s in os.environ.get("RAMBO_SCALE", "served,large").split(",") if s]
FULL = os.environ.get("RAMBO_SCALE_FULL", "") == "1"
ROWS = os.environ.get("RAMBO_SCALE_ROWS", "") == "1"
pytestmark = pytest.mark.gpu
D = 64 if FULL else 256   # every D-th row of every repetition is compared
OUT = os.path.join(os.environ.get("GRAFT_REPO_ROOT", os.path.dirname(os.path.dirname(os.path.abspath(__file__)))),
                   "gpurun_out")

WORKLOADS = {
    # a small stand-in with the served row width, to try the path in seconds
    "mini": dict(sets=lambda: synth.genome_sets(1099, K=2000, n_ancestors=20, ancestor_len=20000, median_len=5000,
                                                min_len=500, max_len=20000),
                 index=dict(K=2000, B=200, R=5, m=1 << 22, eta=2, k=31), seed=2099),
    "served": dict(sets=synth.config_served, index=synth.INDEX_SERVED, seed=2004),
    "large": dict(sets=synth.config_large, index=synth.INDEX_LARGE, seed=2005),
}


def progress(msg):
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "scale_progress.log"), "a") as f:
        f.write("%s %s\n" % (time.strftime("%H:%M:%S"), msg))
    print(msg, flush=True)


def log(rec, **kw):
    rec.update(kw)
    progress(json.dumps(kw))


def device_sampled_rows(g, r, D, chunk_rows=1 << 22):
    """Rows p = 0 mod D of repetition r as [m/D, S/32] uint32 (copied in chunks)."""
    spw = g.row_bits // 32
    out = []
    for p0 in range(0, g.m, chunk_rows):
        n = min(chunk_rows, g.m - p0)
        w = g.index_words(r * g.words_per_rep + p0 * spw, n * spw).view(n, spw)
        out.append(host_u32(w[::D].contiguous()))
        del w
    return np.concatenate(out)


def rows_equal(dev_words, oracle_words, B):
    """Device rows (S/32 uint32 words) against oracle rows (ceil(B/64) uint64
    words): the first B bits equal, the rest of the device row zero."""
    db = np.unpackbits(np.ascontiguousarray(dev_words).view(np.uint8), axis=-1, bitorder="little")
    ob = np.unpackbits(np.ascontiguousarray(oracle_words).view(np.uint8), axis=-1, bitorder="little")
    return np.array_equal(db[..., :B], ob[..., :B]) and not db[..., B:].any()


def scan_rows_chunked(o, sets, D, keys, nthreads, name, pieces=16):
    """orc_scan_rows over the sets in pieces (it ORs into the arrays it is
    given, so the pieces add up to one pass), with a progress line per piece."""
    BW = o.row_words
    sampled = np.zeros((o.R, o.m // D, BW), np.uint64)
    rows = np.zeros((keys.size, BW), np.uint64)
    bounds = np.linspace(0, sets.n, pieces + 1).astype(np.int64)
    lib = oracle.lib()
    t = time.time()
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b <= a:
            continue
        ids = np.ascontiguousarray(sets.set_ids[a:b], np.uint32)
        off = np.ascontiguousarray(sets.offsets[a:b + 1], np.uint64)
        rc = lib.orc_scan_rows(o._h, ids.ctypes.data, off.ctypes.data, sets.chars.ctypes.data, b - a, D,
                               sampled.ctypes.data, keys.ctypes.data, keys.size, rows.ctypes.data, nthreads, 0)
        assert rc == 0
        progress("%s: oracle row scan, sets %d of %d (%.0f s)" % (name, b, sets.n, time.time() - t))
    return sampled, rows


@pytest.fixture(scope="module", params=SCALE)
def workload(request):
    name = request.param
    w = WORKLOADS[name]
    cfg = w["index"]
    rec = {"workload": name, "D": D}
    t = time.time()
    sets = w["sets"]()
    log(rec, sets=int(sets.n), bases=int(sets.chars.size), gen_s=round(time.time() - t, 1))
    g = rb.Rambo(**cfg, seed=w["seed"])
    t = time.time()
    d = (dev(sets.set_ids, np.int32), dev(sets.offsets, np.int64), dev(sets.chars, np.uint8))
    torch.cuda.synchronize()
    h2d = time.time() - t
    n_ins = int(np.maximum(sets.lengths().astype(np.int64) - cfg["k"] + 1, 0).sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.set_timing(True)
    e0.record()
    g.insert_seqs(*d)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    stages = g.stage_times(calls=True)
    g.set_timing(False)
    assert g.sync_status() == rb.OK
    log(rec, index_gib=g.index_bytes / 2**30, inserts=n_ins, insert_ms=ms, inserts_per_s=n_ins / ms * 1e3,
        h2d_s=round(h2d, 1), insert_batches=stages.get("k_bin_regions", (0, 0))[1])
    del d
    torch.cuda.empty_cache()
    o = oracle.OracleIndex(**cfg, seed=w["seed"], flags=oracle.FLAG_NO_FILTERS)
    yield name, cfg, sets, g, o, rec
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "scale_%s.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    g.close()
    o.close()
    torch.cuda.empty_cache()


def device_column(g, r, b, chunk_rows=1 << 22):
    """Bit b of every row of repetition r (the BFU of cell (r, b)) as
    ceil(m/64) uint64 words, bit p of word p/64."""
    spw = g.row_bits // 32
    out = []
    for p0 in range(0, g.m, chunk_rows):
        n = min(chunk_rows, g.m - p0)
        w = g.index_words(r * g.words_per_rep + p0 * spw, n * spw).view(n, spw)[:, b // 32]
        bits = ((w >> (b % 32)) & 1).to(torch.uint8).cpu().numpy()
        out.append(np.packbits(bits, bitorder="little"))
        del w
    return np.concatenate(out).view(np.uint64)


def sampled_reads(name, sets, n_served, n_large):
    if name in ("served", "mini"):
        rq = synth.served_requests(4104, sets, 120)     # about 4 000 reads of 150-5 000 bp
        n_rd = min(rq.n, n_served)
        return synth.SeqBatch(rq.chars[: int(rq.offsets[n_rd])].copy(), rq.offsets[: n_rd + 1].copy(),
                              meta=dict(source_set=rq.meta["source_set"][:n_rd]))
    return synth.reads(3105, sets, n_large, median_len=150, min_len=150, max_len=150, substr_frac=0.8,
                       read_sub_rate=0.01)


def test_scale_cells_and_member_bits(workload):
    name, cfg, sets, g, o, rec = workload
    R, K = cfg["R"], cfg["K"]
    rd = sampled_reads(name, sets, 4000 if FULL else 1000, 10_000 if FULL else 2_000)
    q = synth.kmer_queries(3106, sets, 100_000 if FULL else 10_000, cfg["k"])
    # sampled sets: sources of sampled reads and k-mer queries (answers that
    # hold them), and sets drawn at random (mostly answers that do not)
    rng = np.random.default_rng(3107)
    src_rd, src_q = rd.meta["source_set"], q.meta["source_set"]
    src = sets.set_ids[np.concatenate([src_rd[src_rd >= 0][:5], src_q[src_q >= 0][:2]])].astype(np.int64)
    sample = sorted(set(src.tolist()) | set(rng.integers(0, K, size=3).tolist()))
    phi = o.phi()
    nthreads = min(os.cpu_count() or 1, 16)
    m_rd, nk_rd = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    m_rd, nk_rd = host_u32(m_rd), host_u32(nk_rd)
    id_off, ids, _ = g.query_seqs_ids(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    id_off, ids = id_off.cpu().numpy(), ids.cpu().numpy()
    m_q, _ = g.query_seqs(dev(q.offsets, np.int64), dev(q.chars, np.uint8))
    m_q = host_u32(m_q)
    codes = g.extract_kmers(dev(q.offsets, np.int64), dev(q.chars, np.uint8))
    codes = codes[torch.from_numpy(q.offsets[:-1].astype(np.int64)).cuda()].contiguous()
    m_k = host_u32(g.query_kmers(codes))
    t = time.time()
    cells_done = {}
    n_pos_rd = n_pos_q = 0
    for s in sample:
        cells = []
        for r in range(R):
            b = int(phi[r, s])
            if (r, b) not in cells_done:
                want = o.cell_bits(r, b, sets.set_ids, sets.offsets, sets.chars, nthreads=nthreads)
                assert np.array_equal(device_column(g, r, b), want), "cell (%d, %d)" % (r, b)
                cells_done[(r, b)] = want
            cells.append(cells_done[(r, b)])
        bit = lambda m: ((m[:, s // 32] >> np.uint32(s % 32)) & 1).astype(bool)
        want_rd = o.members_from_cells(rd.offsets, rd.chars, cells)
        assert np.array_equal(bit(m_rd), want_rd), "set %d, reads" % s
        in_ids = np.array([s in ids[id_off[i]:id_off[i + 1]] for i in range(rd.n)])
        assert np.array_equal(in_ids, want_rd), "set %d, ID lists" % s
        want_q = o.members_from_cells(q.offsets, q.chars, cells)
        assert np.array_equal(bit(m_q), want_q), "set %d, k-mers as reads" % s
        assert np.array_equal(bit(m_k), want_q), "set %d, k-mer codes" % s
        n_pos_rd += int(want_rd.sum())
        n_pos_q += int(want_q.sum())
        progress("%s: set %d: %d cells equal, member bits equal (%.0f s)" % (name, s, R, time.time() - t))
    # the k-mers cut from sampled sets are in their answers (no false
    # negatives), so some compared bits are ones; a read with a substitution
    # usually leaves its source's answer
    assert n_pos_q > 0
    for i in range(rd.n):   # ID lists and masks are one answer
        assert ids[id_off[i]:id_off[i + 1]].tolist() == oracle.mask_to_ids(m_rd[i], K)
    log(rec, sampled_sets=sample, cells_compared=len(cells_done), cell_bits_compared=len(cells_done) * cfg["m"],
        member_reads=int(rd.n), member_kmers=int(q.n), positives_reads=n_pos_rd, positives_kmers=n_pos_q,
        cells_s=round(time.time() - t, 1))


def test_scale_rows_and_sampled_answers(workload):
    name, cfg, sets, g, o, rec = workload
    if not ROWS:
        pytest.skip("the full row scan takes minutes of host time: RAMBO_SCALE_ROWS=1 runs it")
    rd = sampled_reads(name, sets, 4000 if FULL else 200, 10_000 if FULL else 1_000)
    q = synth.kmer_queries(3106, sets, 100_000 if FULL else 10_000, cfg["k"])
    keys = np.unique(np.concatenate([o.window_keys(rd.offsets, rd.chars), o.window_keys(q.offsets, q.chars)]))
    nthreads = min(os.cpu_count() or 1, 16)
    t = time.time()
    sampled, rows = scan_rows_chunked(o, sets, D, keys, nthreads, name)
    log(rec, oracle_scan_s=round(time.time() - t, 1), oracle_threads=nthreads, sampled_rows=int(sampled.shape[1]),
        needed_rows=int(keys.size))
    for r in range(cfg["R"]):
        assert rows_equal(device_sampled_rows(g, r, D), sampled[r], cfg["B"]), "repetition %d" % r
    log(rec, sampled_rows_equal=True, rows_compared=int(cfg["R"] * sampled.shape[1]))
    # reads: masks and ID lists against the oracle's answers from rows
    want, wk = o.query_seqs_rows(rd.offsets, rd.chars, keys, rows, nthreads=nthreads)
    m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    assert np.array_equal(host_u32(nk), wk.astype(np.uint32))
    assert np.array_equal(host_u32(m), want)
    id_off, ids, _ = g.query_seqs_ids(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    id_off = id_off.cpu().numpy()
    ids = ids.cpu().numpy()
    for i in range(rd.n):
        assert ids[id_off[i]:id_off[i + 1]].tolist() == oracle.mask_to_ids(want[i], cfg["K"])
    # single k-mers: the read path on one window, and the k-mer path on its code
    qw, _ = o.query_seqs_rows(q.offsets, q.chars, keys, rows, nthreads=nthreads)
    qm, _ = g.query_seqs(dev(q.offsets, np.int64), dev(q.chars, np.uint8))
    assert np.array_equal(host_u32(qm), qw)
    codes = g.extract_kmers(dev(q.offsets, np.int64), dev(q.chars, np.uint8))
    codes = codes[torch.from_numpy(q.offsets[:-1].astype(np.int64)).cuda()].contiguous()
    assert np.array_equal(host_u32(g.query_kmers(codes)), qw)
    log(rec, reads_equal=int(rd.n), kmer_queries_equal=int(q.n),
        mean_answer_sets=float(np.mean([len(oracle.mask_to_ids(x, cfg["K"])) for x in want[:200]])))


def test_scale_no_false_negatives(workload):
    name, cfg, sets, g, o, rec = workload
    rd = synth.reads(3107, sets, 20000, median_len=300, min_len=31, max_len=5000, substr_frac=1.0)
    src = rd.meta["source_set"]
    m, nk = g.query_seqs(dev(rd.offsets, np.int64), dev(rd.chars, np.uint8))
    m = host_u32(m)
    has = (m[np.arange(rd.n), src // 32] >> (src % 32).astype(np.uint32)) & 1
    assert has[host_u32(nk) > 0].all()
    log(rec, no_false_negatives_reads=int((host_u32(nk) > 0).sum()))


def test_scale_serving(workload):
    name, cfg, sets, g, o, rec = workload
    if name not in ("served", "mini"):
        pytest.skip("serving is measured on the served workload")
    n_req = 10_000 if FULL else 2_000
    loads = [0.1, 0.25, 0.4, 0.55, 0.7, 0.85, 1.0, 1.2] if FULL else [0.25, 0.7, 1.0]
    batch = synth.served_requests(4004, sets, n_req)
    reqs = serve.split_requests(batch)
    with rb.Server(g, max_slots=4, use_graphs=True) as srv:
        serve.saturated(srv, reqs[:200], g.W)
        res = serve.sweep_native(srv, batch, loads)
        res["server"] = srv.stats()
    keep = ("load", "offered_qps", "qps", "reads_per_s", "p50_ms", "p99_ms")
    log(rec, serving_saturated={k: res["saturated"][k] for k in ("qps", "reads_per_s", "p50_ms", "p99_ms")},
        serving_points=[{k: p[k] for k in keep} for p in res["points"]], serving_slots=res["server"]["slots"])
    # requests answered in the mix equal the same requests answered alone
    with rb.Server(g, max_slots=4, use_graphs=True) as srv:
        ids = [srv.submit(off, ch) for off, ch in reqs[:300]]
        mixed = [srv.wait(i, len(off) - 1, timeout_us=60_000_000)[0] for i, (off, _) in zip(ids, reqs[:300])]
    for (off, ch), got in zip(reqs[:300], mixed):
        alone, _ = g.query_seqs(dev(off, np.int64), dev(ch, np.uint8))
        assert np.array_equal(host_u32(alone), got)


def test_scale_batched_ids(workload):
    """The large workload's query batch: reads of 150 bp (80% set substrings
    with 1% further substitutions, 20% random), answered as ID lists in one
    call; throughput, the answer-size histogram, and the ID lists against
    the mask form of the same reads."""
    name, cfg, sets, g, o, rec = workload
    if name not in ("large", "mini"):
        pytest.skip("the ID-list batch is the large workload's")
    n = (1_000_000 if FULL else 200_000) if name == "large" else 20_000
    rd = synth.reads(3205, sets, n, median_len=150, min_len=150, max_len=150, substr_frac=0.8, read_sub_rate=0.01)
    off, ch = dev(rd.offsets, np.int64), dev(rd.chars, np.uint8)
    ids_buf = torch.empty(8 << 20, dtype=torch.int32, device="cuda")
    g.query_seqs_ids(off, ch, ids=ids_buf)            # warm-up (and state growth)
    g.set_timing(True)
    g.stage_times()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    id_off, ids, nk = g.query_seqs_ids(off, ch, ids=ids_buf)
    e1.record()
    torch.cuda.synchronize()
    stages = g.stage_times()
    g.set_timing(False)
    ms = e0.elapsed_time(e1)
    sizes = np.diff(id_off.cpu().numpy())
    hist = np.bincount(np.minimum(sizes, 10), minlength=11)
    m, _ = g.query_seqs(off, ch)
    m = host_u32(m)
    ids = ids.cpu().numpy()
    io = id_off.cpu().numpy()
    for i in np.random.default_rng(1).choice(rd.n, size=min(rd.n, 2000), replace=False):
        assert ids[io[i]:io[i + 1]].tolist() == oracle.mask_to_ids(m[i], cfg["K"])
    log(rec, ids_reads=int(rd.n), ids_ms=ms, ids_reads_per_s=rd.n / ms * 1e3,
        ids_kmers_per_s=float(nk.to(torch.int64).sum()) / ms * 1e3, ids_stage_ms=stages,
        ids_total=int(sizes.sum()), answer_size_hist_0_to_10plus=hist.tolist())
