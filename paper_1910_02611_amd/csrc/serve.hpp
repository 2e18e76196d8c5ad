// Continuous-batching query server (include/rambo_serve.h).  Included at the
// end of rambo_api.hip: it uses the handle's internals.
//
// One worker thread owns the index handle while the server runs.  It loops:
// retire finished batches (event query), then fill every free slot with a
// batch of queued requests (host pack into pinned staging, one H2D copy of
// offsets and one of bytes, the three work-queue kernels - replayed from a
// hipGraph captured per slot when asked - and one D2H copy of masks and
// counts), then sleeps briefly only when there is nothing to do.
//
// Device memory: without graphs, every batch takes a region of one device
// pool sized for what it actually holds (its reads' bytes and offsets, K-bit
// masks and per-read state), so a batch is admitted when the pool has room
// for it and frees the room when it retires; with graphs, every slot owns
// fixed buffers for the largest batch (a replayed graph keeps its pointers).  An insert
// request is a barrier in the FIFO: batches stop at it, it runs once every
// earlier batch has finished, and later requests wait for it, so answers are
// those of running the requests one by one in submission order.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "rambo_serve.h"
#include "serve_pool.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct ServeRequest {
    int64_t id = 0;
    uint64_t n_reads = 0;
    std::vector<uint64_t> offsets;   // rebased to 0
    std::vector<uint8_t> chars;
    Clock::time_point t_submit, t_start, t_done;   // submitted, its batch's work enqueued, answered
    std::vector<uint32_t> masks;     // n_reads * W
    std::vector<uint32_t> nk;        // n_reads
    bool done = false;
    bool insert = false;             // an insertion of n_reads sequences into set_ids
    std::vector<uint32_t> set_ids;
    int status = RAMBO_OK;
};

struct ServeSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    void *dmem = nullptr;            // device: header+offsets, bytes, masks, counts, queue state
    uint64_t *d_hdr = nullptr;       // [0] = reads, [1..] = offsets
    uint8_t *d_chars = nullptr;
    uint32_t *d_masks = nullptr;     // device addresses of h_masks, h_nk: the kernels
    uint32_t *d_nk = nullptr;        //   write the answers straight to host memory
    ReadQueue rq{};
    void *hmem = nullptr;            // pinned host: header+offsets, bytes, masks, counts
    uint8_t *hmem_dev = nullptr;     //   the same memory as the device addresses it
    uint64_t *h_hdr = nullptr;
    uint8_t *h_chars = nullptr;
    uint32_t *h_masks = nullptr;
    uint32_t *h_nk = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t region = rambo_pool::kNone;   // the batch's region of the device pool (pool mode)
    uint64_t region_bytes = 0;
    bool busy = false;
    uint64_t n_reads = 0;
    std::vector<std::shared_ptr<ServeRequest>> reqs;
};

}  // namespace

struct rambo_server {
    rambo *h = nullptr;
    rambo_serve_config cfg{};
    std::vector<ServeSlot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<ServeRequest>> queue;
    std::unordered_map<int64_t, std::shared_ptr<ServeRequest>> live;
    int64_t next_id = 0;
    bool stop = false;
    std::thread worker;
    uint64_t n_batches = 0, n_requests = 0, n_reads = 0, n_failed = 0;
    uint32_t inject_failures = 0;     // test hook: batches to fail on the host before they launch
    void *ins_mem = nullptr;          // device staging of insert requests (grown on demand)
    uint64_t ins_cap = 0;
    bool by_bytes = false;            // batches take regions of the pool (no graphs)
    void *pool_mem = nullptr;         // the pool's device memory (mem_budget bytes)
    rambo_pool::Pool pool;            // guarded by mu
    uint64_t mem_waits = 0;           // queued queries that waited for pool room
    int64_t last_waiter = -1;
    // worker timing (microseconds, maxima since the last reset): between two
    // passes of its loop, one batch's enqueue (copies and launches), one
    // completion query
    double max_loop_gap_us = 0, max_enqueue_us = 0, max_query_us = 0;
    bool worker_idle = false;
    int device = 0;
    bool timing_before = false;
};

namespace {

// Copy n_hdr and n_chr 16-byte words from mapped host memory to the
// batch's header and bytes on the device.
__global__ __launch_bounds__(kBlock) void k_pull_batch(const u32x4 *hdr_src, const u32x4 *chr_src, u32x4 *hdr_dst,
                                                       u32x4 *chr_dst, uint64_t n_hdr, uint64_t n_chr)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_hdr + n_chr; i += stride) {
        if (i < n_hdr)
            hdr_dst[i] = hdr_src[i];
        else
            chr_dst[i - n_hdr] = chr_src[i - n_hdr];
    }
}

void free_slot(ServeSlot &s)
{
    if (s.exec)
        (void)hipGraphExecDestroy(s.exec);
    if (s.graph)
        (void)hipGraphDestroy(s.graph);
    if (s.done_ev)
        (void)hipEventDestroy(s.done_ev);
    if (s.stream)
        (void)hipStreamDestroy(s.stream);
    if (s.dmem)
        (void)hipFree(s.dmem);
    if (s.hmem)
        (void)hipHostFree(s.hmem);
    s = ServeSlot{};
}

// Point slot s's device buffers at mem (laid out as batch_layout for
// n_reads reads and n_bytes bytes).
void place_slot(const rambo *h, ServeSlot &s, void *mem, uint64_t n_reads, uint64_t n_bytes)
{
    const rambo_pool::BatchLayout l = rambo_pool::batch_layout(n_reads, n_bytes, read_queue_bytes(h, n_reads));
    uint8_t *d = static_cast<uint8_t *>(mem);
    s.d_hdr = reinterpret_cast<uint64_t *>(d + l.hdr);
    s.d_chars = d + l.chars;
    s.rq = carve_read_queue(h, d + l.state, n_reads);
}

uint64_t batch_device_bytes(const rambo *h, uint64_t n_reads, uint64_t n_bytes)
{
    return rambo_pool::batch_layout(n_reads, n_bytes, read_queue_bytes(h, n_reads)).total;
}

int init_slot(rambo *h, const rambo_serve_config &c, ServeSlot &s, bool own_buffers)
{
    const uint64_t R = c.max_batch_reads;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming) != hipSuccess ||
        (own_buffers && hipMalloc(&s.dmem, batch_device_bytes(h, R, c.max_batch_bytes)) != hipSuccess)) {
        (void)hipGetLastError();
        return RAMBO_ENOMEM;
    }
    // header and bytes 256-aligned (the device pulls them in 16-byte words)
    const uint64_t o_chars = div_up(8 * (R + 2), 256) * 256, o_masks = o_chars + div_up(c.max_batch_bytes, 256) * 256;
    const uint64_t hb = o_masks + 4ull * R * h->W + 4 * R + 64;
    void *dev = nullptr;
    if (hipHostMalloc(&s.hmem, hb, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&dev, s.hmem, 0) != hipSuccess) {
        (void)hipGetLastError();
        return RAMBO_ENOMEM;
    }
    s.hmem_dev = static_cast<uint8_t *>(dev);
    uint8_t *p = static_cast<uint8_t *>(s.hmem);
    s.h_hdr = reinterpret_cast<uint64_t *>(p);
    s.h_chars = p + o_chars;
    p += o_masks;
    s.h_masks = reinterpret_cast<uint32_t *>(p);
    p += 4ull * R * h->W;
    s.h_nk = reinterpret_cast<uint32_t *>(p);
    s.d_masks = reinterpret_cast<uint32_t *>(s.hmem_dev + o_masks);
    s.d_nk = reinterpret_cast<uint32_t *>(s.hmem_dev + o_masks + 4ull * R * h->W);
    if (own_buffers)
        place_slot(h, s, s.dmem, R, c.max_batch_bytes);
    if (own_buffers && c.use_graphs) {
        // the three kernels with the read count taken from device memory
        if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return RAMBO_EHIP;
        launch_read_queue(h, s.rq, s.d_hdr + 1, 0, s.d_hdr, R, s.d_chars, c.max_batch_bytes, s.d_masks, s.d_nk,
                          s.stream);
        if (hipStreamEndCapture(s.stream, &s.graph) != hipSuccess ||
            hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            return RAMBO_EHIP;
        }
    }
    return RAMBO_OK;
}

// Give slot s's pool region back (pool mode; the caller holds mu).
void release_region(rambo_server *sv, ServeSlot &s)
{
    if (s.region != rambo_pool::kNone) {
        sv->pool.release(s.region, s.region_bytes);
        s.region = rambo_pool::kNone;
        s.region_bytes = 0;
    }
}

// Hand every request of slot s back with `status` (a failed batch: no
// answers), and free the slot.
void fail_batch(rambo_server *sv, ServeSlot &s, int status)
{
    const auto t = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (const auto &r : s.reqs) {
            r->masks.assign(r->n_reads * sv->h->W, 0u);
            r->nk.assign(r->n_reads, 0u);
            r->status = status;
            r->t_done = t;
            r->done = true;
        }
        sv->n_failed += 1;
        sv->n_requests += s.reqs.size();
        release_region(sv, s);
    }
    sv->cv_done.notify_all();
    s.reqs.clear();
    s.busy = false;
}

// Pack queued requests into slot s and start its batch.  Called by the
// worker with the lock not held; returns whether a batch was taken (started,
// or failed at once: then its requests are answered with RAMBO_EHIP).
bool start_batch(rambo_server *sv, ServeSlot &s)
{
    const rambo_serve_config &c = sv->cfg;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        uint64_t reads = 0, bytes = 0;
        // pool mode: the largest region free now bounds the batch
        const uint64_t room = sv->by_bytes ? sv->pool.largest_free() : ~0ull;
        const auto at = [&](size_t i) {
            const auto &r = sv->queue[i];
            return rambo_pool::Queued{r->insert, r->n_reads, r->offsets.back()};
        };
        const auto need = [&](uint64_t n, uint64_t b) { return sv->by_bytes ? batch_device_bytes(sv->h, n, b) : 0; };
        // a batch takes at most an equal share of the pool past its first
        // request, so that every slot can run one
        const uint64_t share = sv->by_bytes ? sv->pool.size() / sv->slots.size() : ~0ull;
        const size_t take = rambo_pool::batch_take(sv->queue.size(), at, need, c.max_batch_reads, c.max_batch_bytes,
                                                   room, share, reads, bytes);
        if (take == 0 && !sv->queue.empty() && !sv->queue.front()->insert &&
            sv->queue.front()->id != sv->last_waiter) {
            ++sv->mem_waits;   // admitted when a running batch frees its region
            sv->last_waiter = sv->queue.front()->id;
        }
        for (size_t i = 0; i < take; ++i) {
            s.reqs.push_back(sv->queue.front());
            sv->queue.pop_front();
        }
        if (sv->by_bytes && !s.reqs.empty()) {
            s.region_bytes = batch_device_bytes(sv->h, reads, bytes);
            s.region = sv->pool.alloc(s.region_bytes);   // fits: at most the largest free region
            if (s.region == rambo_pool::kNone) {
                for (auto it = s.reqs.rbegin(); it != s.reqs.rend(); ++it)
                    sv->queue.push_front(*it);
                s.reqs.clear();
                s.region_bytes = 0;
                return false;
            }
            place_slot(sv->h, s, static_cast<uint8_t *>(sv->pool_mem) + s.region, reads, bytes);
        }
    }
    if (s.reqs.empty())
        return false;
    uint64_t reads = 0, bytes = 0;
    for (const auto &r : s.reqs) {
        for (uint64_t i = 0; i < r->n_reads; ++i)
            s.h_hdr[1 + reads + i] = bytes + r->offsets[i];
        std::memcpy(s.h_chars + bytes, r->chars.data(), r->chars.size());
        reads += r->n_reads;
        bytes += r->chars.size();
    }
    s.h_hdr[0] = reads;
    s.h_hdr[1 + reads] = bytes;
    s.n_reads = reads;
    bool injected = false;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->inject_failures) {
            --sv->inject_failures;
            injected = true;
        }
    }
    const auto t_enq = Clock::now();
    hipError_t e = injected ? hipErrorUnknown : hipSuccess;
    if (e == hipSuccess) {
        // header and bytes pulled from the mapped pinned staging by a kernel
        // on the slot's stream, and the answers written back to it by the
        // query kernels: no copy-engine transfers (the enqueue of one of a
        // few hundred KB has been seen to block for 5-10 ms now and then)
        const uint64_t n_hdr = div_up(8 * (reads + 2), 16), n_chr = div_up(bytes, 16);
        const uint32_t grid = (uint32_t)std::min<uint64_t>(div_up(n_hdr + n_chr, kBlock), 1024);
        hipLaunchKernelGGL(k_pull_batch, dim3(grid), dim3(kBlock), 0, s.stream,
                           reinterpret_cast<const u32x4 *>(s.hmem_dev),
                           reinterpret_cast<const u32x4 *>(s.hmem_dev + (s.h_chars - static_cast<uint8_t *>(s.hmem))),
                           reinterpret_cast<u32x4 *>(s.d_hdr), reinterpret_cast<u32x4 *>(s.d_chars), n_hdr, n_chr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        if (s.exec)
            e = hipGraphLaunch(s.exec, s.stream);
        else {
            launch_read_queue(sv->h, s.rq, s.d_hdr + 1, reads, nullptr, reads, s.d_chars, bytes, s.d_masks, s.d_nk,
                              s.stream);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess)
        e = hipEventRecord(s.done_ev, s.stream);
    if (e == hipSuccess) {
        const auto t = Clock::now();
        for (const auto &r : s.reqs)
            r->t_start = t;
        const double us = std::chrono::duration<double, std::micro>(t - t_enq).count();
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->max_enqueue_us = std::max(sv->max_enqueue_us, us);
    }
    if (e != hipSuccess) {
        if (!injected)
            (void)hipGetLastError();
        // whatever was enqueued before the failure must finish before the
        // slot's buffers are reused
        (void)hipStreamSynchronize(s.stream);
        fail_batch(sv, s, RAMBO_EHIP);
        return true;
    }
    s.busy = true;
    return true;
}

void finish_batch(rambo_server *sv, ServeSlot &s)
{
    const auto t = Clock::now();
    const uint32_t W = sv->h->W;
    uint64_t row = 0;
    for (const auto &r : s.reqs) {
        r->masks.assign(s.h_masks + row * W, s.h_masks + (row + r->n_reads) * W);
        r->nk.assign(s.h_nk + row, s.h_nk + row + r->n_reads);
        row += r->n_reads;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (const auto &r : s.reqs) {
            r->t_done = t;
            r->done = true;
        }
        sv->n_batches += 1;
        sv->n_requests += s.reqs.size();
        sv->n_reads += s.n_reads;
        release_region(sv, s);
    }
    sv->cv_done.notify_all();
    s.reqs.clear();
    s.busy = false;
}

// Run insert request r (every earlier batch has finished): stage its data on
// the device, insert with atomics (no scratch), wait, and read the error
// flags.  Returns the request's status.
int run_insert(rambo_server *sv, ServeRequest &r)
{
    rambo *h = sv->h;
    const uint64_t n = r.n_reads, nb = r.chars.size();
    const uint64_t o_off = div_up(4 * n, 256) * 256, o_chars = o_off + div_up(8 * (n + 1), 256) * 256;
    const uint64_t need = o_chars + div_up(nb, 256) * 256;
    if (need > sv->ins_cap) {
        if (sv->ins_mem)
            (void)hipFree(sv->ins_mem);
        sv->ins_cap = 0;
        if (hipMalloc(&sv->ins_mem, need) != hipSuccess) {
            (void)hipGetLastError();
            sv->ins_mem = nullptr;
            return RAMBO_ENOMEM;
        }
        sv->ins_cap = need;
    }
    uint8_t *d = static_cast<uint8_t *>(sv->ins_mem);
    hipStream_t st = sv->slots[0].stream;
    if (hipMemcpyAsync(d, r.set_ids.data(), 4 * n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d + o_off, r.offsets.data(), 8 * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
        (nb && hipMemcpyAsync(d + o_chars, r.chars.data(), nb, hipMemcpyHostToDevice, st) != hipSuccess)) {
        (void)hipGetLastError();
        return RAMBO_EHIP;
    }
    int rc = RAMBO_OK;
    if (nb)
        rc = insert_seqs_direct(h, reinterpret_cast<const uint32_t *>(d), reinterpret_cast<const uint64_t *>(d + o_off),
                                n, d + o_chars, nb, st);
    const int rs = rambo_sync_status(h, st);
    return rc ? rc : rs;
}

void finish_insert(rambo_server *sv, const std::shared_ptr<ServeRequest> &r)
{
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->t_done = Clock::now();
        r->done = true;
        sv->n_requests += 1;
    }
    sv->cv_done.notify_all();
}

void serve_loop(rambo_server *sv)
{
    (void)hipSetDevice(sv->device);   // the current device is per thread
    auto t_pass = Clock::now();
    for (;;) {
        bool progress = false, any_busy = false;
        {
            const auto t = Clock::now();
            const double gap = std::chrono::duration<double, std::micro>(t - t_pass).count();
            t_pass = t;
            bool waited;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                waited = sv->worker_idle;   // a gap spent blocked on an empty queue is not a stall
                sv->worker_idle = false;
                if (!waited)
                    sv->max_loop_gap_us = std::max(sv->max_loop_gap_us, gap);
            }
        }
        for (ServeSlot &s : sv->slots) {
            if (!s.busy)
                continue;
            const auto t_q = Clock::now();
            const hipError_t q = hipEventQuery(s.done_ev);
            {
                const double us = std::chrono::duration<double, std::micro>(Clock::now() - t_q).count();
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->max_query_us = std::max(sv->max_query_us, us);
            }
            if (q == hipSuccess) {
                finish_batch(sv, s);
                progress = true;
            } else if (q != hipErrorNotReady) {
                // the batch failed on the device: its requests get the error
                // instead of waiting for an event that will not complete
                (void)hipGetLastError();
                fail_batch(sv, s, RAMBO_EHIP);
                progress = true;
            }
        }
        for (ServeSlot &s : sv->slots) {
            if (!s.busy && start_batch(sv, s))
                progress = true;
            any_busy = any_busy || s.busy;
        }
        if (!any_busy) {
            std::shared_ptr<ServeRequest> ins;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                if (!sv->queue.empty() && sv->queue.front()->insert) {
                    ins = sv->queue.front();
                    sv->queue.pop_front();
                }
            }
            if (ins) {
                ins->status = run_insert(sv, *ins);
                finish_insert(sv, ins);
                continue;
            }
        }
        if (progress)
            continue;
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stop && sv->queue.empty() && !any_busy)
            return;
        if (any_busy) {
            // batches in flight: look again shortly (or as soon as work arrives)
            sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            sv->worker_idle = true;
        }
    }
}

}  // namespace

extern "C" int rambo_serve_create(rambo_t *h, const rambo_serve_config *cfg_in, rambo_server_t **out)
{
    if (!h || !out)
        return RAMBO_EINVAL;
    *out = nullptr;
    if (const int rr = refuse_raw_keys(h, "rambo_serve_create"))
        return rr;
    rambo_serve_config c = cfg_in ? *cfg_in : rambo_serve_config{};
    if (c.mem_budget == 0)
        c.mem_budget = 1ull << 30;
    if (c.max_batch_bytes == 0)
        c.max_batch_bytes = 8ull << 20;
    if (c.max_slots == 0)
        c.max_slots = 4;
    if (c.max_batch_reads == 0)
        c.max_batch_reads = 8192;
    if (c.max_slots > 16 || c.max_batch_reads > (1u << 24) || c.max_batch_bytes > (1ull << 34))
        return fail(h, RAMBO_EINVAL, "rambo_serve_create: configuration out of range");
    // with graphs, every slot holds buffers for the largest batch; without,
    // the batches share one pool of mem_budget bytes
    const bool by_bytes = !c.use_graphs;
    const uint64_t per_slot = batch_device_bytes(h, c.max_batch_reads, c.max_batch_bytes);
    // (either way the budget must hold one batch of the largest size)
    const uint64_t n_slots = by_bytes ? (c.mem_budget >= per_slot ? c.max_slots : 0)
                                      : std::min<uint64_t>(c.max_slots, c.mem_budget / per_slot);
    if (n_slots == 0)
        return fail(h, RAMBO_ENOMEM, "rambo_serve_create: budget holds no batch of the largest size");
    auto *sv = new (std::nothrow) rambo_server();
    if (!sv)
        return RAMBO_ENOMEM;
    sv->h = h;
    sv->cfg = c;
    sv->by_bytes = by_bytes;
    if (by_bytes) {
        if (hipMalloc(&sv->pool_mem, c.mem_budget) != hipSuccess) {
            (void)hipGetLastError();
            delete sv;
            return fail(h, RAMBO_ENOMEM, "rambo_serve_create: pool allocation failed");
        }
        sv->pool.reset(c.mem_budget);
    }
    sv->slots.resize(n_slots);
    (void)hipGetDevice(&sv->device);
    const bool timing = h->timing;
    sv->timing_before = timing;
    h->timing = false;   // no timing events inside captured graphs or from the worker
    for (ServeSlot &s : sv->slots) {
        const int rc = init_slot(h, c, s, !by_bytes);
        if (rc) {
            for (ServeSlot &t : sv->slots)
                free_slot(t);
            if (sv->pool_mem)
                (void)hipFree(sv->pool_mem);
            delete sv;
            h->timing = timing;
            return fail(h, rc, "rambo_serve_create: slot set-up failed");
        }
    }
    sv->worker = std::thread(serve_loop, sv);
    ++h->servers;
    *out = sv;
    return RAMBO_OK;
}

extern "C" void rambo_serve_destroy(rambo_server_t *sv)
{
    if (!sv)
        return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable())
        sv->worker.join();
    for (ServeSlot &s : sv->slots) {
        if (s.stream)
            (void)hipStreamSynchronize(s.stream);
        free_slot(s);
    }
    if (sv->ins_mem)
        (void)hipFree(sv->ins_mem);
    if (sv->pool_mem)
        (void)hipFree(sv->pool_mem);
    sv->h->timing = sv->timing_before;
    --sv->h->servers;
    delete sv;
}

extern "C" int64_t rambo_serve_submit(rambo_server_t *sv, const uint64_t *offsets, uint64_t n_reads,
                                      const uint8_t *chars)
{
    if (!sv || !offsets || n_reads == 0)
        return RAMBO_EINVAL;
    const uint64_t b0 = offsets[0], b1 = offsets[n_reads];
    if (b1 < b0 || n_reads > sv->cfg.max_batch_reads || b1 - b0 > sv->cfg.max_batch_bytes || (b1 > b0 && !chars))
        return RAMBO_EINVAL;
    if (sv->by_bytes && batch_device_bytes(sv->h, n_reads, b1 - b0) > sv->pool.size())
        return RAMBO_EINVAL;   // would never fit the pool
    auto r = std::make_shared<ServeRequest>();
    r->n_reads = n_reads;
    r->offsets.resize(n_reads + 1);
    for (uint64_t i = 0; i <= n_reads; ++i) {
        const uint64_t o = offsets[i] < b0 ? b0 : (offsets[i] > b1 ? b1 : offsets[i]);
        r->offsets[i] = o - b0;
    }
    if (b1 > b0)
        r->chars.assign(chars + b0, chars + b1);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->id = sv->next_id++;
        r->t_submit = Clock::now();
        sv->live[r->id] = r;
        sv->queue.push_back(r);
    }
    sv->cv_work.notify_one();
    return r->id;
}

extern "C" int64_t rambo_serve_submit_insert(rambo_server_t *sv, const uint32_t *set_ids, const uint64_t *offsets,
                                             uint64_t n_seqs, const uint8_t *chars)
{
    if (!sv || !offsets || !set_ids || n_seqs == 0)
        return RAMBO_EINVAL;
    const uint64_t b0 = offsets[0], b1 = offsets[n_seqs];
    if (b1 < b0 || (b1 > b0 && !chars))
        return RAMBO_EINVAL;
    auto r = std::make_shared<ServeRequest>();
    r->insert = true;
    r->n_reads = n_seqs;
    r->set_ids.assign(set_ids, set_ids + n_seqs);
    r->offsets.resize(n_seqs + 1);
    for (uint64_t i = 0; i <= n_seqs; ++i) {
        const uint64_t o = offsets[i] < b0 ? b0 : (offsets[i] > b1 ? b1 : offsets[i]);
        r->offsets[i] = o - b0;
    }
    if (b1 > b0)
        r->chars.assign(chars + b0, chars + b1);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->id = sv->next_id++;
        r->t_submit = Clock::now();
        sv->live[r->id] = r;
        sv->queue.push_back(r);
    }
    sv->cv_work.notify_one();
    return r->id;
}

namespace {

// rambo_serve_wait, also giving the time from submission to the enqueue of
// the request's batch (queue_ms, if not NULL).
int wait_request(rambo_server_t *sv, int64_t id, uint32_t *masks, uint32_t *nkmers, double *latency_ms,
                 double *queue_ms, int64_t timeout_us)
{
    if (!sv)
        return RAMBO_EINVAL;
    std::shared_ptr<ServeRequest> r;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->live.find(id);
        if (it == sv->live.end())
            return RAMBO_EINVAL;
        r = it->second;
        auto ready = [&] { return r->done; };
        if (timeout_us < 0)
            sv->cv_done.wait(lk, ready);
        else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
            return RAMBO_ETIMEDOUT;
        sv->live.erase(it);
    }
    if (masks)
        std::memcpy(masks, r->masks.data(), r->masks.size() * 4);
    if (nkmers)
        std::memcpy(nkmers, r->nk.data(), r->nk.size() * 4);
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (queue_ms)
        *queue_ms = r->t_start >= r->t_submit
                        ? std::chrono::duration<double, std::milli>(r->t_start - r->t_submit).count() : 0.0;
    return r->status;
}

}  // namespace

extern "C" int rambo_serve_wait(rambo_server_t *sv, int64_t id, uint32_t *masks, uint32_t *nkmers,
                                double *latency_ms, int64_t timeout_us)
{
    return wait_request(sv, id, masks, nkmers, latency_ms, nullptr, timeout_us);
}

extern "C" int rambo_serve_replay(rambo_server_t *sv, uint64_t n_req, const uint64_t *req_reads,
                                  const uint64_t *read_offsets, const uint8_t *chars, const double *arrival_s,
                                  double *latency_ms, double *queue_ms, uint64_t *checksum)
{
    if (!sv || !req_reads || !read_offsets || !arrival_s || !latency_ms)
        return RAMBO_EINVAL;
    for (uint64_t i = 0; i < n_req; ++i)
        if (req_reads[i + 1] < req_reads[i] || req_reads[i + 1] - req_reads[i] > sv->cfg.max_batch_reads ||
            req_reads[i + 1] == req_reads[i] || (i > 0 && arrival_s[i] < arrival_s[i - 1]))
            return RAMBO_EINVAL;
    std::vector<int64_t> ids(n_req, -1);
    std::vector<double> lag(n_req, 0.0);
    std::mutex mu;
    std::condition_variable cv;
    uint64_t submitted = 0;
    int submit_rc = RAMBO_OK;
    const auto t0 = Clock::now() + std::chrono::milliseconds(5);
    std::thread submitter([&] {
        for (uint64_t i = 0; i < n_req; ++i) {
            const auto due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
            std::this_thread::sleep_until(due);
            const auto now = Clock::now();
            const uint64_t a = req_reads[i], n = req_reads[i + 1] - a;
            const int64_t id = rambo_serve_submit(sv, read_offsets + a, n, chars);
            std::lock_guard<std::mutex> lk(mu);
            if (id < 0) {
                submit_rc = (int)id;
                break;
            }
            ids[i] = id;
            lag[i] = now > due ? std::chrono::duration<double, std::milli>(now - due).count() : 0.0;
            submitted = i + 1;
            cv.notify_one();
        }
        std::lock_guard<std::mutex> lk(mu);
        submitted = n_req;   // wakes the collector even after a failed submit
        cv.notify_one();
    });
    const uint32_t W = sv->h->W;
    std::vector<uint32_t> masks, nk;
    uint64_t sum = 0;
    int rc = RAMBO_OK;
    for (uint64_t i = 0; i < n_req; ++i) {
        int64_t id;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return submitted > i; });
            id = ids[i];
        }
        if (id < 0) {
            rc = submit_rc ? submit_rc : RAMBO_EINVAL;
            break;
        }
        const uint64_t n = req_reads[i + 1] - req_reads[i];
        masks.resize(n * W);
        nk.resize(n);
        double ms = 0, qms = 0;
        if ((rc = wait_request(sv, id, masks.data(), nk.data(), &ms, &qms, -1)))
            break;
        latency_ms[i] = ms + lag[i];
        if (queue_ms)
            queue_ms[i] = qms + lag[i];
        for (uint32_t v : masks)
            sum = sum * 1000003u + v;
    }
    submitter.join();
    if (checksum)
        *checksum = sum;
    return rc;
}

extern "C" int rambo_serve_inject_failures(rambo_server_t *sv, uint32_t n_batches)
{
    if (!sv)
        return RAMBO_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->inject_failures = n_batches;
    return RAMBO_OK;
}

extern "C" int rambo_serve_stats(rambo_server_t *sv, uint64_t *batches, uint64_t *requests, uint64_t *reads,
                                 uint32_t *slots)
{
    if (!sv)
        return RAMBO_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (batches)
        *batches = sv->n_batches;
    if (requests)
        *requests = sv->n_requests;
    if (reads)
        *reads = sv->n_reads;
    if (slots)
        *slots = (uint32_t)sv->slots.size();
    return RAMBO_OK;
}

extern "C" int rambo_serve_worker_stats(rambo_server_t *sv, double *max_loop_gap_us, double *max_enqueue_us,
                                        double *max_query_us, int reset)
{
    if (!sv)
        return RAMBO_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (max_loop_gap_us)
        *max_loop_gap_us = sv->max_loop_gap_us;
    if (max_enqueue_us)
        *max_enqueue_us = sv->max_enqueue_us;
    if (max_query_us)
        *max_query_us = sv->max_query_us;
    if (reset)
        sv->max_loop_gap_us = sv->max_enqueue_us = sv->max_query_us = 0;
    return RAMBO_OK;
}

extern "C" uint64_t rambo_serve_batch_bytes(const rambo_t *h, uint64_t n_reads, uint64_t n_bytes)
{
    return h ? batch_device_bytes(h, n_reads, n_bytes) : 0;
}

extern "C" int rambo_serve_mem_stats(rambo_server_t *sv, uint64_t *budget, uint64_t *in_use, uint64_t *peak,
                                     uint64_t *waits)
{
    if (!sv)
        return RAMBO_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    const uint64_t fixed = sv->by_bytes ? 0 : batch_device_bytes(sv->h, sv->cfg.max_batch_reads,
                                                                  sv->cfg.max_batch_bytes) * sv->slots.size();
    if (budget)
        *budget = sv->by_bytes ? sv->pool.size() : fixed;
    if (in_use)
        *in_use = sv->by_bytes ? sv->pool.used() : fixed;
    if (peak)
        *peak = sv->by_bytes ? sv->pool.peak() : fixed;
    if (waits)
        *waits = sv->mem_waits;
    return RAMBO_OK;
}
