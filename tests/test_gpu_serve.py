"""The query server (include/rambo_serve.h): every request's answer is the
oracle's, and the same whether the request ran alone or packed into a batch
with others, with or without captured graphs, over one or several slots."""
import threading

import numpy as np
import pytest

from paper_1910_02611_amd import rambo as rb
from paper_1910_02611_amd import serve, synth
import oracle
from gpu_util import make_pair, gpu_insert_seqs

pytestmark = pytest.mark.gpu
TIMEOUT_US = 30_000_000   # a lost request fails the test instead of hanging it


@pytest.fixture(scope="module")
def served():
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o, g = make_pair(cfg, seed=2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    gpu_insert_seqs(g, sets)
    batch = synth.served_requests(4010, sets, 80, max_len=1500)
    reqs = serve.split_requests(batch)
    # edge requests: empty read, reads shorter than k, a break in every window
    edge_chars = np.frombuffer(b"ACG" + b"A" * 31 + b"ACGTNACGTACGTACGTACGTACGTACGTACGTAC", np.uint8)
    edge_off = np.array([0, 0, 3, 34, 34 + 35], np.uint64)
    reqs.insert(5, (edge_off, edge_chars))
    want = []
    for off, ch in reqs:
        m, nk = o.query_seqs(off, ch, nthreads=8)
        want.append((m, nk.astype(np.uint32)))
    return g, reqs, want


def check(got, want):
    for i, ((m, nk), (wm, wn)) in enumerate(zip(got, want)):
        assert np.array_equal(nk, wn), i
        assert np.array_equal(m, wm), i


def alone(srv, reqs):
    out = []
    for off, ch in reqs:
        rid = srv.submit(off, ch)
        m, nk, _ = srv.wait(rid, len(off) - 1, timeout_us=TIMEOUT_US)
        out.append((m, nk))
    return out


def mixed(srv, reqs, lead=None):
    """Submit everything before waiting for anything (after an optional
    large leading request that keeps the first slot busy meanwhile)."""
    lead_id = srv.submit(*lead) if lead is not None else None
    ids = [srv.submit(off, ch) for off, ch in reqs]
    out = [srv.wait(rid, len(off) - 1, timeout_us=TIMEOUT_US)[:2] for rid, (off, _) in zip(ids, reqs)]
    if lead_id is not None:
        srv.wait(lead_id, len(lead[0]) - 1, timeout_us=TIMEOUT_US)
    return out


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("slots", [1, 4])
def test_alone_and_mixed_match_oracle(served, graphs, slots):
    g, reqs, want = served
    with rb.Server(g, max_slots=slots, use_graphs=graphs, max_batch_reads=256, max_batch_bytes=1 << 20) as srv:
        a = alone(srv, reqs)
        check(a, want)
        m = mixed(srv, reqs)
        check(m, want)
        st = srv.stats()
    assert st["requests"] == 2 * len(reqs)
    assert st["reads"] == 2 * sum(len(off) - 1 for off, _ in reqs)


def test_requests_share_batches(served):
    g, reqs, want = served
    # a large first request keeps the only slot busy while the rest queue up
    rng = np.random.default_rng(7)
    big_chars = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=4000 * 2000)
    big_off = np.arange(0, 4000 * 2000 + 1, 2000, dtype=np.uint64)
    with rb.Server(g, max_slots=1, max_batch_reads=4096, max_batch_bytes=16 << 20) as srv:
        m = mixed(srv, reqs, lead=(big_off, big_chars))
        st = srv.stats()
    check(m, want)
    assert st["requests"] == len(reqs) + 1
    assert st["batches"] < st["requests"]   # some batch held several requests


def test_concurrent_clients(served):
    g, reqs, want = served
    got = [None] * len(reqs)

    def client(c):
        for i in range(c, len(reqs), 4):
            off, ch = reqs[i]
            rid = srv.submit(off, ch)
            got[i] = srv.wait(rid, len(off) - 1, timeout_us=TIMEOUT_US)[:2]

    with rb.Server(g, max_slots=3, use_graphs=True, max_batch_reads=512) as srv:
        ts = [threading.Thread(target=client, args=(c,)) for c in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    check(got, want)


def test_open_loop_driver(served):
    g, reqs, want = served
    with rb.Server(g, max_slots=2) as srv:
        r = serve.run_open_loop(srv, reqs, synth.poisson_arrivals(9, len(reqs), 2000.0), g.W)
    assert r["requests"] == len(reqs)
    assert 0 < r["p50_ms"] <= r["p99_ms"]


def test_errors(served):
    g, reqs, _ = served
    with rb.Server(g, max_slots=1, max_batch_reads=16, max_batch_bytes=4096) as srv:
        off = np.arange(0, 17 * 10 + 1, 10, dtype=np.uint64)   # 17 reads
        with pytest.raises(rb.RamboError):   # more reads than a batch holds
            srv.submit(off, np.zeros(170, np.uint8))
        with pytest.raises(rb.RamboError):   # more bytes than a batch holds
            srv.submit(np.array([0, 5000], np.uint64), np.zeros(5000, np.uint8))
        with pytest.raises(rb.RamboError):   # unknown id
            srv.wait(12345, 1, timeout_us=0)
    for graphs in (False, True):
        with pytest.raises(rb.RamboError):    # budget too small for one batch of the largest size
            rb.Server(g, mem_budget=1024, use_graphs=graphs)


def test_admission_by_device_bytes(served):
    # a pool that holds about one batch of the largest size: batches are
    # sized by what their requests hold, so several small ones run at once,
    # and requests wait in the queue for room; answers stay the oracle's
    g, reqs, want = served
    # room for one batch of 64 reads and 128 KiB (the largest request is
    # 96 KB), so at most a few single-request batches at once for 16 slots
    budget = rb.lib().rambo_serve_batch_bytes(g._h, 64, 128 << 10)
    assert budget > 0
    with rb.Server(g, max_slots=16, mem_budget=budget, max_batch_reads=64, max_batch_bytes=128 << 10) as srv:
        m = mixed(srv, reqs)
        st = srv.stats()
    check(m, want)
    assert st["mem_budget"] == budget // 256 * 256
    assert 0 < st["mem_peak"] <= st["mem_budget"] and st["mem_in_use"] == 0
    assert st["mem_waits"] > 0 and st["batches"] > 1


@pytest.mark.parametrize("use_graphs", [False, True])
def test_streaming_inserts_between_queries(use_graphs):
    """Inserts submitted between queries (streaming updates, Sec. 3.1) take
    effect in submission order: queries before the k-th insert equal the
    oracle with the first k-1 insert batches, queries after it the oracle
    with k, however the requests are batched."""
    cfg = dict(K=64, B=8, R=3, eta=2, k=31, m=1 << 18)
    sets = synth.genome_sets(4100, K=64, n_ancestors=8, ancestor_len=4000, median_len=2000, min_len=500,
                             max_len=4000)
    o, g = make_pair(cfg, seed=77)
    parts = np.array_split(np.arange(sets.n), 3)     # three insert batches
    reqs = serve.split_requests(synth.served_requests(4101, sets, 30, max_len=1500))
    phases = []
    with rb.Server(g, max_slots=3, use_graphs=use_graphs) as srv:
        ids = []
        for k, part in enumerate(parts):
            sub_off = np.concatenate([[0], np.cumsum(sets.lengths()[part])]).astype(np.uint64)
            sub_chars = np.concatenate([sets.chars[int(sets.offsets[i]):int(sets.offsets[i + 1])] for i in part])
            ids.append(("q", k, [srv.submit(off, ch) for off, ch in reqs]))
            ids.append(("i", k, srv.submit_insert(sets.set_ids[part], sub_off, sub_chars)))
        ids.append(("q", len(parts), [srv.submit(off, ch) for off, ch in reqs]))
        for kind, k, rid in ids:
            if kind == "i":
                assert srv.wait_insert(rid, timeout_us=TIMEOUT_US) >= 0
            else:
                phases.append([srv.wait(r, len(off) - 1, timeout_us=TIMEOUT_US)[:2] for r, (off, _) in zip(rid, reqs)])
        # a bad set id: the insert reports it, the server goes on
        bad = srv.submit_insert(np.array([cfg["K"]], np.uint32), np.array([0, 40], np.uint64),
                                np.frombuffer(b"ACGT" * 10, np.uint8))
        with pytest.raises(rb.RamboError) as e:
            srv.wait_insert(bad, timeout_us=TIMEOUT_US)
        assert e.value.code == rb.ERANGE
        after = srv.wait(srv.submit(*reqs[0]), len(reqs[0][0]) - 1, timeout_us=TIMEOUT_US)[:2]
    for k, got in enumerate(phases):
        if k > 0:
            part = parts[k - 1]
            assert o.insert_seqs(sets.set_ids[part], np.concatenate([[0], np.cumsum(sets.lengths()[part])]),
                                 np.concatenate([sets.chars[int(sets.offsets[i]):int(sets.offsets[i + 1])]
                                                 for i in part]), 8) == 0
        want = []
        for off, ch in reqs:
            m, nk = o.query_seqs(off, ch, nthreads=8)
            want.append((m, nk.astype(np.uint32)))
        check(got, want)
    check([after], [want[0]])


def _checksum(masks_in_order):
    s = 0
    for m in masks_in_order:
        for v in np.asarray(m, dtype=np.uint32).reshape(-1).tolist():
            s = (s * 1000003 + v) & ((1 << 64) - 1)
    return s


def test_native_replay_driver(served):
    """rambo_serve_replay submits the requests from a native thread at their
    arrival times; its checksum over every answer word equals the oracle's
    answers in request order, saturated and paced."""
    g, _, _ = served
    cfg = synth.INDEX_TINY
    sets = synth.config_tiny()
    o = oracle.OracleIndex(cfg["K"], cfg["B"], cfg["R"], cfg["eta"], cfg["k"], cfg["m"], 2001)
    o.insert_seqs(sets.set_ids, sets.offsets, sets.chars, 8)
    batch = synth.served_requests(4020, sets, 60, max_len=1500)
    ro = batch.meta["request_offsets"]
    want = []
    for r in range(ro.size - 1):
        off, ch = synth.request(batch, r)
        want.append(o.query_seqs(off, ch, nthreads=8)[0])
    with rb.Server(g, max_slots=3, use_graphs=True) as srv:
        for arrivals in (np.zeros(ro.size - 1), synth.poisson_arrivals(7, ro.size - 1, 2000.0)):
            lat, ck, qms = srv.replay(ro, batch.offsets, batch.chars, arrivals, with_queue=True)
            assert ck == _checksum(want)
            assert (lat > 0).all() and (qms >= 0).all() and (qms <= lat).all()
        bad = ro.copy()
        bad[1] = bad[0]            # a request without reads
        with pytest.raises(rb.RamboError):
            srv.replay(bad, batch.offsets, batch.chars, np.zeros(ro.size - 1))


@pytest.mark.parametrize("graphs", [False, True])
def test_failed_batches_answer_with_an_error(served, graphs):
    # the worker's error path, forced from the host (no device fault): the
    # requests of a failed batch are answered with RAMBO_EHIP instead of
    # blocking their waiters, and the server goes on answering later ones
    g, reqs, want = served
    with rb.Server(g, max_slots=2, use_graphs=graphs) as srv:
        srv.inject_failures(1)
        rid = srv.submit(*reqs[0])
        with pytest.raises(rb.RamboError) as e:
            srv.wait(rid, len(reqs[0][0]) - 1, timeout_us=TIMEOUT_US)
        assert e.value.code == rb.EHIP
        check(alone(srv, reqs[:10]), want[:10])
        srv.inject_failures(3)
        ids = [srv.submit(off, ch) for off, ch in reqs[:20]]
        codes = []
        for rid, (off, _) in zip(ids, reqs[:20]):
            try:
                srv.wait(rid, len(off) - 1, timeout_us=TIMEOUT_US)
                codes.append(rb.OK)
            except rb.RamboError as err:
                codes.append(err.code)
        assert set(codes) <= {rb.OK, rb.EHIP} and rb.EHIP in codes
        check(alone(srv, reqs[:10]), want[:10])
