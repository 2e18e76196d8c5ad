// Host runtime and C ABI of the RAMBO index (declared in include/rambo.h).
//
// The handle owns the bit-sliced index, the partition table phi, the cell
// membership masks and a sticky device error word.  Every call checks its
// arguments on the host, then enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "insert_part.hpp"
#include "insert_pieces.hpp"
#include "query_ids.hpp"
#include "query_queue.hpp"
#include "kernels.hpp"
#include "rambo.h"

using namespace rambo_dev;

struct rambo {
    rambo_config cfg{};
    Params P{};
    uint32_t S = 0, SW = 0, W = 0;
    uint64_t words_per_rep = 0;
    uint64_t index_bytes = 0;
    uint32_t *index = nullptr;
    uint16_t *phi = nullptr;
    uint32_t *cellmask = nullptr;
    uint32_t *member_off = nullptr;   // R x (B+1)
    uint32_t *members = nullptr;      // R x K
    int *err = nullptr;
    bool index_zero = true;          // nothing inserted since create or clear
    std::string last_error;
    // partitioned insertion
    int insert_mode = RAMBO_INSERT_AUTO;
    uint64_t scratch_limit = 0;      // 0: chosen at first use
    rambo_insert_tiles tiles{};      // requested tile shapes of the partitioned insert (0 = automatic)
    bool part_ok = false;            // geometry supports the partitioned path
    BinGeom bin{};
    uint64_t bin_targets = 0;        // targets per batch the scratch holds
    void *bin_mem = nullptr;
    uint32_t piece_nwg = 0;          // workgroups of the piece kernel (stage A for sequences)
    uint64_t piece_capA = 0;         // entries of each of its chunks the scratch holds
    uint32_t *piece_mem = nullptr;   // first piece of each sequence (n_seqs + 1 words)
    uint64_t piece_cap = 0;
    // batched sequence queries
    int query_mode = RAMBO_QUERY_AUTO;
    uint32_t query_chunk = 512;        // bytes per work item
    uint32_t query_waves_per_cu = 16;  // persistent grid
    int num_cus = 256;
    void *rq_mem = nullptr;
    uint64_t rq_cap = 0;               // reads the queue state holds
    int servers = 0;                   // query servers attached (their graphs hold index pointers)
    bool recorded_insert = false;      // an insert was recorded into a graph: index_zero is never trusted again
    ReadQueue rq{};
    uint64_t *scan_part = nullptr;     // tile totals of the ID-list scan (in rq_mem)
    void *noalloc = nullptr;           // this GPU's scratch of rambo_query_seqs_ids_noalloc
    std::string noalloc_error;         //   or why it could not be found
    bool rq_recorded = false;          // a captured graph holds rq_mem: retire it instead of freeing it
    std::vector<void *> retired;       // scratch buffers captured graphs may still use; freed by rambo_destroy
    // ordering of the handle's scratch across streams: the last call that
    // used it recorded scratch_ev on scratch_stream
    hipEvent_t scratch_ev = nullptr;
    hipStream_t scratch_stream = nullptr;
    bool scratch_pending = false;
    // kernel timing (rambo_set_timing)
    bool timing = false;
    mutable std::vector<hipEvent_t> ev_pool;
    mutable size_t ev_used = 0;
    struct Stage {
        const char *name;
        hipEvent_t a, b;
    };
    mutable std::vector<Stage> stages;
};

namespace {

// Brackets one kernel launch with two events on its stream when timing is on.
// Whether work on stream st is being recorded into a graph (then nothing
// runs now: host-side state must not assume the work has happened, and no
// timing events are recorded).
bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// The index is no longer known to be zero; an insert recorded into a graph
// may run later unseen by the host, so from then on it never is.
void note_insert(rambo *h, hipStream_t stream)
{
    h->index_zero = false;
    if (capturing(stream))
        h->recorded_insert = true;
}

// The handle's scratch (insert slabs, read-queue state) is shared by every
// call, whatever its stream: a call on a stream other than the previous
// scratch user's first waits for that user's work (an event recorded at the
// end of each such call), so calls on different streams never overlap in the
// scratch.  Work recorded into a graph is ordered by the graph instead.
struct ScratchUse {
    rambo *h;
    hipStream_t st;
    ScratchUse(rambo *h_, hipStream_t st_) : h(h_), st(st_)
    {
        if (h->scratch_pending && st != h->scratch_stream && h->scratch_ev && !capturing(st))
            (void)hipStreamWaitEvent(st, h->scratch_ev, 0);
    }
    ~ScratchUse()
    {
        if (!h->scratch_ev || capturing(st))
            return;
        if (hipEventRecord(h->scratch_ev, st) == hipSuccess) {
            h->scratch_stream = st;
            h->scratch_pending = true;
        } else {
            (void)hipGetLastError();
        }
    }
};

struct StageScope {
    const rambo *h;
    hipStream_t st;
    hipEvent_t b = nullptr;
    StageScope(const rambo *h_, const char *name, hipStream_t st_) : h(h_), st(st_)
    {
        if (!h->timing || h->stages.size() >= 100000 || capturing(st))
            return;
        hipEvent_t ev[2];
        for (hipEvent_t &e : ev) {
            if (h->ev_used == h->ev_pool.size()) {
                hipEvent_t n = nullptr;
                if (hipEventCreate(&n) != hipSuccess)
                    return;
                h->ev_pool.push_back(n);
            }
            e = h->ev_pool[h->ev_used++];
        }
        (void)hipEventRecord(ev[0], st);
        b = ev[1];
        h->stages.push_back({name, ev[0], ev[1]});
    }
    ~StageScope()
    {
        if (b)
            (void)hipEventRecord(b, st);
    }
};

}  // namespace

namespace {

thread_local std::string g_create_error;

constexpr uint64_t kP61 = (1ull << 61) - 1;
constexpr uint64_t kChunk = 1024;   // bytes per wave in the window walkers

uint64_t splitmix64_next(uint64_t &state)
{
    state += 0x9E3779B97F4A7C15ull;
    return mix64(state);
}

int fail(rambo *h, int code, const std::string &msg)
{
    if (h)
        h->last_error = msg;
    else
        g_create_error = msg;
    return code;
}

int hip_check(rambo *h, hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return RAMBO_OK;
    return fail(h, RAMBO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int launch_check(rambo *h, const char *what)
{
    return hip_check(h, hipGetLastError(), what);
}

uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- dispatch

template <int SW, int R_T, int ETA_T>
void launch_query_kmers_t(const rambo *h, const uint64_t *codes, uint64_t n, uint32_t *out, hipStream_t st)
{
    constexpr int G = SW > 4 ? SW / 4 : 1;
    constexpr uint64_t QPB = kBlock / G;
    StageScope sc(h, "k_query_kmers", st);
    hipLaunchKernelGGL((k_query_kmers<SW, R_T, ETA_T>), dim3((uint32_t)div_up(n, QPB)), dim3(kBlock), 0, st, h->P,
                       codes, n, out);
}

template <int SW, int R_T, int ETA_T>
void launch_query_seqs_t(const rambo *h, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars,
                         uint64_t n_chars, uint32_t *out, uint32_t *nk, const ReadQueue &rq, hipStream_t st)
{
    StageScope sc(h, "k_query_seqs", st);
    hipLaunchKernelGGL((k_query_seqs<SW, R_T, ETA_T>), dim3((uint32_t)div_up(n_reads, kWavesPerBlock)),
                       dim3(kBlock), 0, st, h->P, offsets, n_reads, chars, n_chars, out, nk, rq.G, rq.nk, rq.dead);
}

// Row widths of the workloads get kernels with compile-time R and eta (all
// gathers of a term in flight at once); everything else takes the run-time
// path.
template <int SW>
constexpr bool kSpecialised = SW == 1 || SW == 2 || SW == 8 || SW == 32;

template <int SW, class F>
void with_shape(const rambo *h, F &&f)
{
    const uint32_t R = h->cfg.R, E = h->cfg.eta;
    if constexpr (kSpecialised<SW>) {
        if (E == 2) {
            switch (R) {
            case 3: f.template operator()<SW, 3, 2>(); return;
            case 4: f.template operator()<SW, 4, 2>(); return;
            case 5: f.template operator()<SW, 5, 2>(); return;
            case 6: f.template operator()<SW, 6, 2>(); return;
            default: break;
            }
        }
    }
    if constexpr (SW == 64) {
        if (E == 4 && R == 2) {   // the word-unigram index of Sec. 5.3 (B = 2000)
            f.template operator()<64, 2, 4>();
            return;
        }
    }
    f.template operator()<SW, 0, 0>();
}

template <class F>
void with_row_words(const rambo *h, F &&f)
{
    switch (h->SW) {
    case 1: with_shape<1>(h, f); break;
    case 2: with_shape<2>(h, f); break;
    case 4: with_shape<4>(h, f); break;
    case 8: with_shape<8>(h, f); break;
    case 16: with_shape<16>(h, f); break;
    case 32: with_shape<32>(h, f); break;
    case 64: with_shape<64>(h, f); break;
    default: with_shape<128>(h, f); break;
    }
}

struct QueryKmersLaunch {
    const rambo *h;
    const uint64_t *codes;
    uint64_t n;
    uint32_t *out;
    hipStream_t st;
    template <int SW, int R_T, int ETA_T>
    void operator()() const { launch_query_kmers_t<SW, R_T, ETA_T>(h, codes, n, out, st); }
};

template <int SW, int R_T, int ETA_T>
void launch_query_termsets_t(const rambo *h, const uint64_t *offsets, uint64_t n_sets, const uint64_t *codes,
                             uint64_t n_codes, uint32_t *out, hipStream_t st)
{
    StageScope sc(h, "k_query_termsets", st);
    constexpr uint64_t SPB = (uint64_t)kWavesPerBlock * termsets_per_wave<SW, R_T>();
    hipLaunchKernelGGL((k_query_termsets<SW, R_T, ETA_T>), dim3((uint32_t)div_up(n_sets, SPB)), dim3(kBlock), 0, st,
                       h->P, offsets, n_sets, codes, n_codes, out);
}

struct QueryTermsetsLaunch {
    const rambo *h;
    const uint64_t *offsets;
    uint64_t n_sets;
    const uint64_t *codes;
    uint64_t n_codes;
    uint32_t *out;
    hipStream_t st;
    template <int SW, int R_T, int ETA_T>
    void operator()() const { launch_query_termsets_t<SW, R_T, ETA_T>(h, offsets, n_sets, codes, n_codes, out, st); }
};

struct QuerySeqsLaunch {
    const rambo *h;
    const uint64_t *offsets;
    uint64_t n_reads;
    const uint8_t *chars;
    uint64_t n_chars;
    uint32_t *out;
    uint32_t *nk;
    hipStream_t st;
    const ReadQueue &rq;   // per-read state, written where out is NULL
    template <int SW, int R_T, int ETA_T>
    void operator()() const
    {
        launch_query_seqs_t<SW, R_T, ETA_T>(h, offsets, n_reads, chars, n_chars, out, nk, rq, st);
    }
};

// The persistent work-queue launch (k_rq_persist); its per-read state is
// already set up by k_rq_setup and k_rq_scan.
struct QuerySeqsQueueLaunch {
    const rambo *h;
    const ReadQueue &rq;
    const uint64_t *offsets;
    uint64_t n_reads;
    const uint64_t *n_dev;
    const uint8_t *chars;
    uint64_t n_chars;
    uint32_t *out;
    uint32_t *nk;
    hipStream_t st;
    uint32_t grid;
    template <int SW, int R_T, int ETA_T>
    void operator()() const
    {
        StageScope sc(h, "k_rq_persist", st);
        hipLaunchKernelGGL((k_rq_persist<SW, R_T, ETA_T>), dim3(grid), dim3(kBlock), 0, st, h->P, rq, offsets,
                           n_reads, n_dev, chars, n_chars, h->query_chunk, out, nk);
    }
};

constexpr int kMaxDevices = 64;
void *noalloc_scratch(int dev, std::string *err);

uint32_t next_pow2(uint32_t v)
{
    uint32_t p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

uint32_t log2_exact(uint64_t v)
{
    uint32_t l = 0;
    while ((1ull << l) < v)
        ++l;
    return l;
}

// Insert kernels with compile-time R and eta for the shapes of the
// workloads, the run-time kernel for every other shape.
using InsertSeqsFn = void (*)(Params, const uint32_t *, const uint64_t *, uint64_t, const uint8_t *, uint64_t,
                              uint64_t);
using BinWindowsFn = void (*)(Params, BinGeom, const uint32_t *, const uint64_t *, uint64_t, const uint8_t *,
                              uint64_t, uint64_t, uint64_t, uint32_t, uint32_t);

template <class Fn, template <int, int> class K>
Fn pick_shape(uint32_t R, uint32_t eta)
{
    if (eta == 2) {
        switch (R) {
        case 3: return K<3, 2>::fn;
        case 4: return K<4, 2>::fn;
        case 5: return K<5, 2>::fn;
        case 6: return K<6, 2>::fn;
        default: break;
        }
    }
    return K<0, 0>::fn;
}

template <int R_T, int ETA_T>
struct InsertSeqsK {
    static constexpr InsertSeqsFn fn = k_insert_seqs<R_T, ETA_T>;
};
template <int R_T, int ETA_T>
struct BinWindowsK {
    static constexpr BinWindowsFn fn = k_bin_windows<R_T, ETA_T>;
};

using BinHoldFn = void (*)(Params, BinGeom, const uint32_t *, const uint64_t *, uint64_t, const uint8_t *, uint64_t,
                           uint64_t, uint64_t, uint32_t);

// Stage A with the targets held in registers, for the compile-time shapes.
BinHoldFn pick_bin_hold(uint32_t R, uint32_t eta)
{
    if (eta == 2) {
        switch (R) {
        case 3: return k_bin_windows_hold<3, 2>;
        case 4: return k_bin_windows_hold<4, 2>;
        case 5: return k_bin_windows_hold<5, 2>;
        case 6: return k_bin_windows_hold<6, 2>;
        default: break;
        }
    }
    return nullptr;
}

using BinCodesFn = void (*)(Params, BinGeom, const uint32_t *, const uint64_t *, uint64_t, const uint64_t *, uint64_t,
                            uint64_t, uint32_t);

// Stage A from codes or raw keys, for the compile-time shapes (those of the
// sequence path and R = 2, eta = 4 of the documents index).
BinCodesFn pick_bin_codes_hold(uint32_t R, uint32_t eta)
{
    if (eta == 2) {
        switch (R) {
        case 3: return k_bin_codes_hold<3, 2>;
        case 4: return k_bin_codes_hold<4, 2>;
        case 5: return k_bin_codes_hold<5, 2>;
        case 6: return k_bin_codes_hold<6, 2>;
        default: break;
        }
    }
    if (eta == 4 && R == 2)
        return k_bin_codes_hold<2, 4>;
    return nullptr;
}

using BinCodesGenFn = void (*)(Params, BinGeom, const uint32_t *, const uint64_t *, uint64_t, const uint64_t *,
                               uint64_t, uint64_t, uint32_t, uint32_t);

// The stage-A kernel from codes of a shape: held targets where compiled,
// else the run-time kernel; its steps per round and LDS bytes.
struct StageACodes {
    BinCodesFn hold = nullptr;
    BinCodesGenFn generic = nullptr;
    uint32_t steps = 0;
    size_t lds = 0;
    const void *fn() const
    {
        return hold ? reinterpret_cast<const void *>(hold) : reinterpret_cast<const void *>(generic);
    }
};

// The stage-A kernel of a shape, its steps per round and its LDS bytes.
struct StageA {
    BinWindowsFn generic = nullptr;
    BinHoldFn hold = nullptr;
    uint32_t steps = 0;
    size_t lds = 0;
};

StageA stage_a(const rambo *h)
{
    const uint32_t RE = h->cfg.R * h->cfg.eta;
    StageA a;
    a.hold = h->bin.na <= kHoldBucketsPerThread * kBlockP ? pick_bin_hold(h->cfg.R, h->cfg.eta) : nullptr;
    if (a.hold) {
        a.steps = hold_steps(RE);
        a.lds = lds_bytes_stage_a_hold(RE, h->bin.na);
    } else {
        a.generic = pick_shape<BinWindowsFn, BinWindowsK>(h->cfg.R, h->cfg.eta);
        a.steps = kTileA / (kBlockP * RE);
        a.lds = lds_bytes_stage_a(h->bin.na);
    }
    return a;
}

StageACodes stage_a_codes(const rambo *h)
{
    const uint32_t RE = h->cfg.R * h->cfg.eta;
    StageACodes a;
    a.hold = h->bin.na <= kHoldBucketsPerThread * kBlockP ? pick_bin_codes_hold(h->cfg.R, h->cfg.eta) : nullptr;
    if (a.hold) {
        a.steps = hold_steps(RE);
        a.lds = lds_bytes_stage_a_hold(RE, h->bin.na);
    } else {
        a.generic = k_bin_codes;
        a.steps = kTileA / (kBlockP * RE);
        a.lds = lds_bytes_stage_a(h->bin.na);
    }
    return a;
}

// ------------------------------------------------ batched read queries

// Per-read state of the work-queue launch, grown to hold n_reads reads.
uint64_t read_queue_bytes(const rambo *h, uint64_t cap)
{
    const uint64_t rsw = (uint64_t)h->cfg.R * h->SW;
    return 4 * (cap * (rsw + 4) + (cap + 1) + 1);
}

// Lay out the per-read state of cap reads in mem (read_queue_bytes(h, cap)).
ReadQueue carve_read_queue(const rambo *h, void *mem, uint64_t cap)
{
    const uint64_t rsw = (uint64_t)h->cfg.R * h->SW;
    ReadQueue q{};
    uint32_t *p = static_cast<uint32_t *>(mem);
    q.G = p;
    p += cap * rsw;
    q.nk = p;
    p += cap;
    q.dead = p;
    p += cap;
    q.remaining = p;
    p += cap;
    q.items = p;
    p += cap + 1;
    q.counter = p;
    return q;
}

int ensure_read_queue(rambo *h, uint64_t n_reads)
{
    if (n_reads <= h->rq_cap && h->rq_mem)
        return RAMBO_OK;
    uint64_t cap = h->rq_cap ? h->rq_cap : 1024;
    while (cap < n_reads)
        cap *= 2;
    if (h->rq_mem) {
        const int rc = hip_check(h, hipDeviceSynchronize(), "read queue resize");
        if (rc)
            return rc;
        if (h->rq_recorded)
            h->retired.push_back(h->rq_mem);   // a captured graph may still replay on it
        else
            (void)hipFree(h->rq_mem);
        h->rq_mem = nullptr;
        h->rq_cap = 0;
        h->rq_recorded = false;
    }
    const uint64_t qb = div_up(read_queue_bytes(h, cap), 256) * 256;
    if (hipMalloc(&h->rq_mem, qb + 8 * (div_up(cap, kScanTile) + 1)) != hipSuccess) {
        (void)hipGetLastError();
        h->rq_mem = nullptr;
        return fail(h, RAMBO_ENOMEM, "read queue allocation failed");
    }
    h->rq = carve_read_queue(h, h->rq_mem, cap);
    h->scan_part = reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(h->rq_mem) + qb);
    h->rq_cap = cap;
    return RAMBO_OK;
}

// One wave per read, or the work queue: as set by rambo_set_query_policy;
// automatically, one wave per read unless reads are long on average (then
// splitting them into chunks balances the load).
constexpr uint64_t kWaveReadMaxMeanBytes = 2048;

bool wave_per_read(const rambo *h, uint64_t n_reads, uint64_t n_chars)
{
    if (h->query_mode != RAMBO_QUERY_AUTO)
        return h->query_mode == RAMBO_QUERY_WAVE_PER_READ;
    return n_chars <= kWaveReadMaxMeanBytes * n_reads;
}

// The three launches of the work-queue read query.  The batch has n_host
// reads, or *n_dev reads (at most cap_reads) when n_dev is given; n_chars
// bounds the byte buffer.
void launch_read_queue(rambo *h, const ReadQueue &rq, const uint64_t *offsets, uint64_t n_host,
                       const uint64_t *n_dev, uint64_t cap_reads, const uint8_t *chars, uint64_t n_chars,
                       uint32_t *out, uint32_t *nk, hipStream_t stream)
{
    const uint32_t rsw = h->cfg.R * h->SW;
    {
        StageScope sc(h, "k_rq_setup", stream);
        hipLaunchKernelGGL(k_rq_setup, dim3((uint32_t)div_up(cap_reads, kBlock)), dim3(kBlock), 0, stream, rq, offsets,
                           n_host, n_dev, n_chars, h->query_chunk, rsw);
    }
    {
        StageScope sc(h, "k_rq_scan", stream);
        hipLaunchKernelGGL(k_rq_scan, dim3(1), dim3(1024), 0, stream, rq.items, n_host, n_dev);
    }
    const uint64_t max_items = n_chars / h->query_chunk + cap_reads + 1;
    const uint64_t waves = std::min<uint64_t>(max_items, (uint64_t)h->num_cus * h->query_waves_per_cu);
    const uint32_t grid = (uint32_t)div_up(waves, kWavesPerBlock);
    with_row_words(h, QuerySeqsQueueLaunch{h, rq, offsets, n_host, n_dev, chars, n_chars, out, nk, stream, grid});
}

// ------------------------------------------------- partitioned insertion

constexpr uint32_t kRegionLog2 = kRegionLog2Max;   // 128 KiB of LDS per region
constexpr uint32_t kMaxCoarse = 4096;       // stage-A LDS: tile plus 3 words per coarse bucket
constexpr size_t kMaxLds = 160 * 1024;      // LDS per workgroup on gfx950
constexpr double kAtomicRate = 1.7e10;      // measured random atomicOr/s over a large buffer
constexpr double kStreamRate = 4.0e12;      // streaming bytes/s the partitioned path sustains
constexpr uint32_t kStageAWindowsPerWave = 2048;

// Regions of 2^rb bits that hold index bits (the last may be partial).
uint64_t n_regions(const BinGeom &G) { return div_up(G.total_words * 32, 1ull << G.rb); }

// Regions of the group of coarse buckets that starts at c0.
uint64_t group_regions(const BinGeom &G, uint32_t c0, uint32_t ncb)
{
    const uint64_t first = (uint64_t)c0 * G.nf, all = n_regions(G);
    return first >= all ? 0 : std::min((uint64_t)ncb * G.nf, all - first);
}

// Stage B's kernel: a tile of about 16 entries per region (runs of a
// 64-byte segment on average) whose LDS fits; the larger tiles take
// workgroups of 1024 threads (4 waves per SIMD at one workgroup per CU) to
// keep a tile's entries in registers.  Measured: at 2048 regions per coarse
// bucket the 32768-entry tile takes 13% less time than the 8192-entry one,
// at 256 regions 5% more.
using BinRegionsFn = void (*)(Params, BinGeom, uint32_t);
struct StageB {
    BinRegionsFn fn;
    int blk;
    uint32_t tile;
    size_t lds;
};

StageB stage_b(const BinGeom &G, uint32_t want = 0)
{
    if (want == 32768 && lds_bytes_stage_b_t<1024, 32768>(G.nf) <= kMaxLds)
        return {k_bin_regions<1024, 32768>, 1024, 32768, lds_bytes_stage_b_t<1024, 32768>(G.nf)};
    if (want == 16384 && lds_bytes_stage_b_t<1024, 16384>(G.nf) <= kMaxLds)
        return {k_bin_regions<1024, 16384>, 1024, 16384, lds_bytes_stage_b_t<1024, 16384>(G.nf)};
    if (want == kTileB)
        return {k_bin_regions<kBlockP, kTileB>, kBlockP, kTileB, lds_bytes_stage_b_t<kBlockP, kTileB>(G.nf)};
    if (G.nf >= 2048 && lds_bytes_stage_b_t<1024, 32768>(G.nf) <= kMaxLds)
        return {k_bin_regions<1024, 32768>, 1024, 32768, lds_bytes_stage_b_t<1024, 32768>(G.nf)};
    if (G.nf >= 1024 && lds_bytes_stage_b_t<1024, 16384>(G.nf) <= kMaxLds)
        return {k_bin_regions<1024, 16384>, 1024, 16384, lds_bytes_stage_b_t<1024, 16384>(G.nf)};
    return {k_bin_regions<kBlockP, kTileB>, kBlockP, kTileB, lds_bytes_stage_b_t<kBlockP, kTileB>(G.nf)};
}

void plan_partition(rambo *h)
{
    const uint64_t total_words = (uint64_t)h->cfg.R * h->words_per_rep;
    const uint64_t total_bits = total_words * 32;
    BinGeom &G = h->bin;
    G.rb = kRegionLog2;
    // Regions per coarse bucket: as many as stage B's largest tile serves
    // with runs of 16 (2^11) while at least 256 coarse buckets remain, then
    // more (to 2^12) while a stage-A round (automatic steps) would give a
    // bucket fewer than 32 entries: with shorter runs the open 128-byte line
    // each workgroup keeps per bucket no longer stays in an XCD's L2 between
    // rounds.  Measured on the 96 GiB insert: 768 -> 384 coarse buckets took
    // stage A from 87.6 to 72.9 ms per launch.
    auto coarse = [&](uint32_t fb) { return div_up(total_bits, 1ull << (G.rb + fb)); };
    const uint64_t round_targets = (uint64_t)(h->cfg.R <= 5 ? 2 : 1) * kBlockPc * h->cfg.R * h->cfg.eta;
    G.fb = 8;
    while (G.fb < 11 && coarse(G.fb + 1) >= 256)
        ++G.fb;
    while (G.fb < 12 && coarse(G.fb) * 32 > round_targets)
        ++G.fb;
    if (h->tiles.fine_bits)
        G.fb = h->tiles.fine_bits;
    G.nf = 1u << G.fb;
    const uint64_t na = div_up(total_bits, 1ull << (G.rb + G.fb));
    G.na = (uint32_t)na;
    G.nwg = 1;
    G.c0 = 0;
    G.ncb = G.na;
    G.total_words = total_words;
    h->part_ok = na <= kMaxCoarse && (uint64_t)h->cfg.R * h->cfg.eta <= kMaxTargetsPerWindow &&
                 lds_bytes_stage_a(G.na) <= kMaxLds && lds_bytes_stage_b(G.nf) <= kMaxLds;
}

// Stage A over sequence pieces for the compiled shapes: the kernel, its LDS
// bytes and how many of its workgroups fit a CU (at most two); it runs as
// that many persistent workgroups per CU.
using BinPiecesFn = void (*)(Params, BinGeom, PieceArgs);
struct StageAPieces {
    BinPiecesFn fn = nullptr;
    size_t lds = 0;
    uint32_t per_cu = 0;
    uint32_t steps = 0;
};

template <int R_T, int ETA_T, int ST>
StageAPieces make_pieces(uint32_t na, bool fast)
{
    StageAPieces a;
    a.lds = lds_bytes_pieces<R_T, ETA_T, ST>(na);
    // one persistent workgroup per CU: measured faster than two on the
    // 8 GiB index (fewer chunks written at once)
    a.per_cu = a.lds <= kMaxLds ? 1u : 0u;
    a.lds = std::max<size_t>(a.lds, kMaxLds / 2 + 1024);
    a.steps = ST;
    if (a.per_cu)
        a.fn = fast ? k_bin_pieces<R_T, ETA_T, ST, true> : k_bin_pieces<R_T, ETA_T, ST, false>;
    return a;
}

StageAPieces stage_a_pieces(const rambo *h)
{
    const BinGeom &G = h->bin;
    const uint32_t shA = G.rb + G.fb;
    const uint64_t rep_bits = h->words_per_rep * 32;
    // 32-bit positions and buckets: m a power of two <= 2^32, repetitions
    // made of whole coarse buckets, and a row no wider than a coarse bucket
    const bool fast = h->P.m_log2 > 0 && h->P.m_log2 <= 32 && shA <= 31 && rep_bits % (1ull << shA) == 0 &&
                      h->P.S_log2 <= shA;
    if (h->cfg.eta == 2 && G.na <= kMaxCoarse) {
        // automatic: two steps per round for R <= 5 where the tile fits LDS
        uint32_t st = h->tiles.steps ? h->tiles.steps : (h->cfg.R <= 5 ? 2u : 1u);
        if (!h->tiles.steps && st == 2) {
            const size_t lds2 = h->cfg.R == 3 ? lds_bytes_pieces<3, 2, 2>(G.na)
                                : h->cfg.R == 4 ? lds_bytes_pieces<4, 2, 2>(G.na) : lds_bytes_pieces<5, 2, 2>(G.na);
            if (lds2 > kMaxLds)
                st = 1;
        }
        switch (h->cfg.R * 10 + st) {
        case 31: return make_pieces<3, 2, 1>(G.na, fast);
        case 32: return make_pieces<3, 2, 2>(G.na, fast);
        case 41: return make_pieces<4, 2, 1>(G.na, fast);
        case 42: return make_pieces<4, 2, 2>(G.na, fast);
        case 51: return make_pieces<5, 2, 1>(G.na, fast);
        case 52: return make_pieces<5, 2, 2>(G.na, fast);
        case 61: return make_pieces<6, 2, 1>(G.na, fast);
        case 62: return make_pieces<6, 2, 2>(G.na, fast);
        default: break;
        }
    }
    return StageAPieces{};
}

// Slab capacities for T targets per batch spread evenly over the index (the
// index may hold fewer bits than na coarse buckets of nf regions), with
// margins for the statistical spread; skewed inputs overflow into the
// fallback atomics.  capA1: one chunk per coarse bucket (the stage-A kernels
// that reserve runs with atomics); capAn: each of nwg producers' chunk of a
// bucket (the piece kernel); capB: per region.  Stages B and C run over
// groups of ncb coarse buckets, so slab B holds only one group's regions.
struct ScratchPlan {
    uint64_t capA1 = 0, capAn = 0, capB = 0, bytes = 0;
};

uint64_t chunk_cap(const BinGeom &G, uint64_t T, uint32_t nwg)
{
    const double coarse = (double)G.total_words * 32.0 / (double)(1ull << (G.rb + G.fb));
    return div_up((uint64_t)((double)T / (coarse < 1.0 ? 1.0 : coarse) / nwg * 1.04) + 64, 16) * 16;
}

ScratchPlan scratch_plan(const BinGeom &G, uint64_t T, uint32_t nwg, uint32_t ncb)
{
    const double bits = (double)G.total_words * 32.0;
    const double coarse = bits / (double)(1ull << (G.rb + G.fb)), regions = bits / (double)(1ull << G.rb);
    ScratchPlan s;
    s.capA1 = div_up((uint64_t)((double)T / (coarse < 1.0 ? 1.0 : coarse) * 1.04) + 4096, 4) * 4;
    s.capAn = nwg ? chunk_cap(G, T, nwg) : 0;
    s.capB = div_up((uint64_t)((double)T / (regions < 1.0 ? 1.0 : regions) * 1.08) + 512, 4) * 4;
    const uint64_t slabA = std::max((uint64_t)G.na * s.capA1, (uint64_t)G.na * nwg * s.capAn);
    const uint64_t gr = group_regions(G, 0, ncb);
    s.bytes = 4 * (slabA + gr * s.capB + gr + (uint64_t)G.na * G.nf +
                   (uint64_t)G.na * std::max(nwg, 1u));
    return s;
}

// Allocate the scratch of the partitioned path once: as many targets per
// batch as fit the limit.  Each batch's stage C rewrites every region it
// touches, so an insert larger than one batch sweeps the index once per
// batch: the default limit is most of the free memory (85% of what is left
// after keeping kScratchKeepFree free for the caller's query buffers), at
// most kScratchMax.
constexpr uint64_t kScratchKeepFree = 8ull << 30;
constexpr uint64_t kScratchMax = 192ull << 30;

int ensure_scratch(rambo *h, uint64_t want_targets)
{
    if (h->bin_mem)
        return RAMBO_OK;
    uint64_t limit = h->scratch_limit;
    if (limit == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
            return fail(h, RAMBO_EHIP, "hipMemGetInfo failed");
        limit = free_b > 2 * kScratchKeepFree ? (free_b - kScratchKeepFree) / 20 * 19 : free_b / 2;
        if (limit > kScratchMax)
            limit = kScratchMax;
    }
    const StageAPieces AP = stage_a_pieces(h);
    h->piece_nwg = AP.fn ? AP.per_cu * (uint32_t)h->num_cus : 0u;
    const uint64_t want = std::max<uint64_t>(want_targets, 1ull << 24);
    const uint64_t t_max = std::min<uint64_t>(want, 1ull << 35);
    // For 1, 2, 4, 8 groups of coarse buckets in stages B and C: the most
    // targets per batch that fit the limit (slab positions and fill
    // counters are 32-bit).  Take the fewest groups that need the fewest
    // batches: every batch rewrites the index regions it touches once.
    const BinGeom &G0 = h->bin;
    uint64_t best_T = 0, best_batches = ~0ull;
    uint32_t best_ncb = G0.na;
    for (uint32_t ng = 1; ng <= 8 && ng <= G0.na; ng *= 2) {
        if (h->tiles.groups && ng != std::min(h->tiles.groups, G0.na))
            continue;
        const uint32_t ncb = (G0.na + ng - 1) / ng;
        auto fits = [&](uint64_t T) {
            const ScratchPlan p = scratch_plan(G0, T, h->piece_nwg, ncb);
            return p.bytes <= limit && p.capA1 < (1ull << 31) && p.capB < (1ull << 31);
        };
        if (!fits(4096))
            continue;
        uint64_t lo = 4096, hi = t_max;   // fits(lo); find the largest T that fits
        if (fits(hi))
            lo = hi;
        while (hi - lo > 4096) {
            const uint64_t mid = lo + (hi - lo) / 2;
            (fits(mid) ? lo : hi) = mid;
        }
        const uint64_t batches = div_up(want, lo);
        if (batches < best_batches) {
            best_batches = batches;
            best_T = lo;
            best_ncb = ncb;
        }
    }
    if (best_T == 0)
        return fail(h, RAMBO_ENOMEM, "insert scratch limit too small");
    const uint64_t T = best_T;
    const ScratchPlan sp = scratch_plan(G0, T, h->piece_nwg, best_ncb);
    if (hipMalloc(&h->bin_mem, sp.bytes) != hipSuccess) {
        (void)hipGetLastError();
        h->bin_mem = nullptr;
        return fail(h, RAMBO_ENOMEM, "insert scratch allocation failed");
    }
    BinGeom &G = h->bin;
    // stages A, B and C use more than the default 64 KiB of dynamic LDS
    const StageA A = stage_a(h);
    const void *binA = A.hold ? reinterpret_cast<const void *>(A.hold) : reinterpret_cast<const void *>(A.generic);
    const StageACodes AC = stage_a_codes(h);
    if (hipFuncSetAttribute(binA, hipFuncAttributeMaxDynamicSharedMemorySize, (int)A.lds) != hipSuccess ||
        hipFuncSetAttribute(AC.fn(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)AC.lds) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_apply_regions), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((1u << (G.rb - 5)) * 4)) != hipSuccess ||
        (AP.fn && hipFuncSetAttribute(reinterpret_cast<const void *>(AP.fn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)AP.lds) != hipSuccess) ||
        hipFuncSetAttribute(reinterpret_cast<const void *>(stage_b(G, h->tiles.stage_b_tile).fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)stage_b(G, h->tiles.stage_b_tile).lds) != hipSuccess) {
        (void)hipFree(h->bin_mem);
        h->bin_mem = nullptr;
        return fail(h, RAMBO_EHIP, "cannot raise the LDS limit of the insert kernels");
    }
    G.capA = sp.capA1;
    G.capB = sp.capB;
    G.nwg = 1;
    G.c0 = 0;
    G.ncb = best_ncb;
    const uint64_t slabA = std::max((uint64_t)G.na * sp.capA1, (uint64_t)G.na * h->piece_nwg * sp.capAn);
    uint32_t *p = static_cast<uint32_t *>(h->bin_mem);
    G.slabA = p;
    p += slabA;
    G.slabB = p;
    p += group_regions(G, 0, G.ncb) * sp.capB;
    G.fillB = p;
    p += group_regions(G, 0, G.ncb);
    G.dirty = p;
    p += (uint64_t)G.na * G.nf;
    G.fillA = p;   // na * max(nwg, 1); the first na follow dirty, so one fill kernel clears all three
    h->bin_targets = T;
    h->piece_capA = sp.capAn;
    return RAMBO_OK;
}

// Per-sequence piece starts of the piece kernel: n_seqs + 1 words, grown on
// demand (a buffer a captured insert may still replay on is kept).
int ensure_pieces(rambo *h, uint64_t n_seqs)
{
    if (n_seqs + 1 <= h->piece_cap && h->piece_mem)
        return RAMBO_OK;
    uint64_t cap = std::max<uint64_t>(h->piece_cap * 2, 1024);
    while (cap < n_seqs + 1)
        cap *= 2;
    if (h->piece_mem) {
        const int rc = hip_check(h, hipDeviceSynchronize(), "piece table resize");
        if (rc)
            return rc;
        if (h->recorded_insert)
            h->retired.push_back(h->piece_mem);
        else
            (void)hipFree(h->piece_mem);
        h->piece_mem = nullptr;
        h->piece_cap = 0;
    }
    if (hipMalloc(&h->piece_mem, cap * 4) != hipSuccess) {
        (void)hipGetLastError();
        h->piece_mem = nullptr;
        return fail(h, RAMBO_ENOMEM, "piece table allocation failed");
    }
    h->piece_cap = cap;
    return RAMBO_OK;
}

bool use_partitioned(const rambo *h, uint64_t n_chars)
{
    if (!h->part_ok || h->insert_mode == RAMBO_INSERT_DIRECT)
        return false;
    if (h->insert_mode == RAMBO_INSERT_PARTITIONED || h->insert_mode == RAMBO_INSERT_PARTITIONED_WALKER)
        return true;
    const double T = (double)n_chars * h->cfg.R * h->cfg.eta;
    const double regions = (double)h->bin.na * h->bin.nf;
    const double t_direct = T / kAtomicRate;
    const double t_part = (T * 20.0 + (T < regions ? T : regions) * 2.0 * (1u << (kRegionLog2 - 3))) / kStreamRate +
                          100e-6;
    return t_part < t_direct;
}

// Stages B and C of one batch, after its stage A filled slab A as G says:
// one pair of launches per group of G.ncb coarse buckets (slab B holds one
// group's regions; its fill counters are cleared between groups).
void launch_stages_bc(rambo *h, const BinGeom &G, uint32_t fresh, hipStream_t stream)
{
    const StageB SB = stage_b(G, h->tiles.stage_b_tile);
    const uint32_t tpb = (uint32_t)div_up((uint64_t)G.nwg * G.capA, SB.tile);
    const size_t ldsC = (1ull << (G.rb - 5)) * 4;
    for (uint32_t c0 = 0; c0 < G.na; c0 += G.ncb) {
        BinGeom Gg = G;
        Gg.c0 = c0;
        const uint32_t ncb = std::min(G.ncb, G.na - c0);
        Gg.ncb = ncb;   // stage B's grid rounds the group up to whole rounds of XCDs and skips the rest
        const uint64_t regions = group_regions(G, c0, ncb);
        if (c0 > 0) {
            StageScope sc(h, "k_zero_u32", stream);
            hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(kBlock), 0, stream, G.fillB, regions);
        }
        { StageScope sc(h, "k_bin_regions", stream);
        hipLaunchKernelGGL(SB.fn, dim3((uint32_t)(div_up(ncb, kXcds) * kXcds * tpb)), dim3(SB.blk), SB.lds, stream,
                           h->P, Gg, tpb); }
        { StageScope sc(h, "k_apply_regions", stream);
        hipLaunchKernelGGL(k_apply_regions, dim3((uint32_t)regions), dim3(kBlockC), ldsC, stream, h->P, Gg, fresh); }
    }
}

void clear_fill_counters(rambo *h, const BinGeom &G, hipStream_t stream)
{
    StageScope sc(h, "k_zero_u32", stream);
    hipLaunchKernelGGL(k_zero_u32, dim3(1024), dim3(kBlock), 0, stream, G.fillB,
                       group_regions(G, 0, G.ncb) + (uint64_t)G.na * G.nf + G.na);   // fillB, dirty, fillA[0..na)
}

// Stages A to C for codes or raw keys, in batches of the scratch's capacity.
int insert_kmers_partitioned(rambo *h, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_sets,
                             const uint64_t *codes, uint64_t n_codes, hipStream_t stream)
{
    const uint64_t RE = (uint64_t)h->cfg.R * h->cfg.eta;
    int rc = ensure_scratch(h, n_codes * RE);
    if (rc)
        return rc;
    const BinGeom &G = h->bin;
    const StageACodes A = stage_a_codes(h);
    const uint64_t batch = h->bin_targets / RE;
    const uint32_t steps = A.steps;
    const uint32_t rounds = (uint32_t)div_up(kStageAWindowsPerWave, (uint64_t)steps * kWave);
    const uint64_t block_codes = (uint64_t)kWavesP * rounds * steps * kWave;
    // as for sequences: only the first batch into an index known to be all
    // zero skips reading the regions back
    uint32_t fresh = h->index_zero && !h->recorded_insert && !capturing(stream) ? 1u : 0u;
    note_insert(h, stream);
    for (uint64_t p = 0; p < n_codes; p += batch, fresh = 0) {
        const uint64_t pe = p + batch < n_codes ? p + batch : n_codes;
        clear_fill_counters(h, G, stream);
        { StageScope sc(h, "k_bin_codes", stream);
        const dim3 grid((uint32_t)div_up(pe - p, block_codes));
        if (A.hold)
            hipLaunchKernelGGL(A.hold, grid, dim3(kBlockP), A.lds, stream, h->P, G, set_ids, offsets, n_sets, codes,
                               p, pe, rounds);
        else
            hipLaunchKernelGGL(A.generic, grid, dim3(kBlockP), A.lds, stream, h->P, G, set_ids, offsets, n_sets,
                               codes, p, pe, steps, rounds); }
        launch_stages_bc(h, G, fresh, stream);
        if ((rc = launch_check(h, "rambo_insert_kmers (partitioned)")))
            return rc;
    }
    return RAMBO_OK;
}

// Stages A to C for sequences with the piece kernel: pieces are counted and
// numbered on the device, then taken in batches of the scratch's capacity
// (the host knows only an upper bound of the number of pieces; batches past
// the real end find nothing to do).
int insert_seqs_pieces(rambo *h, const StageAPieces &AP, const uint32_t *set_ids, const uint64_t *offsets,
                       uint64_t n_seqs, const uint8_t *chars, uint64_t n_chars, hipStream_t stream)
{
    const uint64_t RE = (uint64_t)h->cfg.R * h->cfg.eta;
    const uint64_t q_up = n_chars / kPieceWindows + n_seqs + 1;
    int rc = ensure_scratch(h, q_up * kPieceWindows * RE);
    if (rc)
        return rc;
    if ((rc = ensure_pieces(h, n_seqs)))
        return rc;
    const uint32_t nwg = h->piece_nwg;
    uint64_t bp = std::max<uint64_t>(1, h->bin_targets / (kPieceWindows * RE));
    const uint64_t nb = div_up(q_up, bp);
    bp = div_up(q_up, nb);
    BinGeom G = h->bin;
    G.nwg = nwg;
    // a batch of at least one piece may hold more targets than the scratch
    // was sized for: its chunks keep their allocated size and the excess
    // goes to the fallback atomics
    G.capA = std::min(chunk_cap(h->bin, bp * kPieceWindows * RE, nwg), h->piece_capA);
    const uint32_t mis = (uint32_t)(reinterpret_cast<uintptr_t>(chars) & 3u);
    PieceArgs pa{set_ids, offsets, n_seqs, chars - mis, n_chars + mis, mis, h->piece_mem, 0, 0};
    {
        StageScope sc(h, "k_piece_counts", stream);
        hipLaunchKernelGGL(k_piece_counts, dim3((uint32_t)div_up(n_seqs, kBlock)), dim3(kBlock), 0, stream, offsets,
                           n_seqs, n_chars, h->cfg.k, h->piece_mem);
        hipLaunchKernelGGL(k_rq_scan, dim3(1), dim3(1024), 0, stream, h->piece_mem, n_seqs, nullptr);
    }
    uint32_t fresh = h->index_zero && !h->recorded_insert && !capturing(stream) ? 1u : 0u;
    note_insert(h, stream);
    for (uint64_t q = 0; q < q_up; q += bp, fresh = 0) {
        pa.q_begin = q;
        pa.q_end = std::min(q + bp, q_up);
        clear_fill_counters(h, G, stream);
        { StageScope sc(h, "k_bin_pieces", stream);
        hipLaunchKernelGGL(AP.fn, dim3(nwg), dim3(kBlockPc), AP.lds, stream, h->P, G, pa); }
        launch_stages_bc(h, G, fresh, stream);
        if ((rc = launch_check(h, "rambo_insert_seqs (partitioned)")))
            return rc;
    }
    return RAMBO_OK;
}

int insert_seqs_partitioned(rambo *h, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_seqs,
                            const uint8_t *chars, uint64_t n_chars, hipStream_t stream)
{
    const StageAPieces AP = stage_a_pieces(h);
    if (AP.fn && h->insert_mode != RAMBO_INSERT_PARTITIONED_WALKER)
        return insert_seqs_pieces(h, AP, set_ids, offsets, n_seqs, chars, n_chars, stream);
    const uint64_t RE = (uint64_t)h->cfg.R * h->cfg.eta;
    int rc = ensure_scratch(h, n_chars * RE);
    if (rc)
        return rc;
    const BinGeom &G = h->bin;
    const uint64_t batch_windows = h->bin_targets / RE;
    // stage A: each round takes `steps` steps of every wave
    const StageA A = stage_a(h);
    const uint32_t steps = A.steps;
    const uint32_t rounds = (uint32_t)div_up(kStageAWindowsPerWave, (uint64_t)steps * kWave);
    const uint64_t block_windows = (uint64_t)kWavesP * rounds * steps * kWave;
    // the first batch into an all-zero index need not read the regions back
    // (never in a captured graph: a replay may find the index holding bits;
    // and never once a recorded insert may have run unseen by the host)
    uint32_t fresh = h->index_zero && !h->recorded_insert && !capturing(stream) ? 1u : 0u;
    note_insert(h, stream);
    for (uint64_t p = 0; p < n_chars; p += batch_windows, fresh = 0) {
        const uint64_t pe = p + batch_windows < n_chars ? p + batch_windows : n_chars;
        clear_fill_counters(h, G, stream);
        { StageScope sc(h, "k_bin_windows", stream);
        const dim3 grid((uint32_t)div_up(pe - p, block_windows));
        if (A.hold)
            hipLaunchKernelGGL(A.hold, grid, dim3(kBlockP), A.lds, stream, h->P, G, set_ids, offsets, n_seqs, chars,
                               n_chars, p, pe, rounds);
        else
            hipLaunchKernelGGL(A.generic, grid, dim3(kBlockP), A.lds, stream, h->P, G, set_ids, offsets, n_seqs,
                               chars, n_chars, p, pe, steps, rounds); }
        launch_stages_bc(h, G, fresh, stream);
        if ((rc = launch_check(h, "rambo_insert_seqs (partitioned)")))
            return rc;
    }
    return RAMBO_OK;
}

// SetIDs(M[b,r]) as ascending member lists (a counting sort of phi_r per
// repetition, on the host, once): the ID-list kernels enumerate candidate
// sets from them.
int build_member_lists(rambo *h)
{
    const uint32_t K = h->cfg.K, B = h->cfg.B, R = h->cfg.R;
    std::vector<uint16_t> phi((size_t)R * K);
    std::vector<uint32_t> off((size_t)R * (B + 1)), mem((size_t)R * K);
    int rc = hip_check(h, hipMemcpy(phi.data(), h->phi, phi.size() * 2, hipMemcpyDeviceToHost), "member lists");
    if (rc)
        return rc;
    for (uint32_t r = 0; r < R; ++r) {
        uint32_t *o = off.data() + (size_t)r * (B + 1);
        const uint16_t *f = phi.data() + (size_t)r * K;
        for (uint32_t i = 0; i < K; ++i)
            ++o[f[i] + 1];
        for (uint32_t b = 0; b < B; ++b)
            o[b + 1] += o[b];
        std::vector<uint32_t> cur(o, o + B);
        for (uint32_t i = 0; i < K; ++i)   // ascending i: each list comes out sorted
            mem[(size_t)r * K + cur[f[i]]++] = i;
    }
    if (hipMalloc(&h->member_off, off.size() * 4) != hipSuccess || hipMalloc(&h->members, mem.size() * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, RAMBO_ENOMEM, "member lists: device allocation failed");
    }
    if ((rc = hip_check(h, hipMemcpy(h->member_off, off.data(), off.size() * 4, hipMemcpyHostToDevice), "member lists")) ||
        (rc = hip_check(h, hipMemcpy(h->members, mem.data(), mem.size() * 4, hipMemcpyHostToDevice), "member lists")))
        return rc;
    h->P.member_off = h->member_off;
    h->P.members = h->members;
    return RAMBO_OK;
}

// SetIDs tables from the current phi and B: the cell masks (zeroed, then
// k_build_cellmask) and the member lists.  Synchronous.
int rebuild_tables(rambo *h)
{
    const rambo_config &c = h->cfg;
    if (h->member_off)
        (void)hipFree(h->member_off);
    if (h->members)
        (void)hipFree(h->members);
    h->member_off = h->members = nullptr;
    int rc = hip_check(h, hipMemset(h->cellmask, 0, (uint64_t)c.R * c.B * h->W * 4), "tables");
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_build_cellmask, dim3((uint32_t)div_up((uint64_t)c.R * h->W, kBlock)), dim3(kBlock), 0, 0,
                       h->phi, c.K, c.B, c.R, h->W, h->cellmask);
    if ((rc = launch_check(h, "tables")) || (rc = hip_check(h, hipDeviceSynchronize(), "tables")))
        return rc;
    return build_member_lists(h);
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" int rambo_create(const rambo_config *cfg, rambo_t **out)
{
    if (!out)
        return fail(nullptr, RAMBO_EINVAL, "rambo_create: out is NULL");
    *out = nullptr;
    if (!cfg)
        return fail(nullptr, RAMBO_EINVAL, "rambo_create: cfg is NULL");
    const rambo_config c = *cfg;
    if (c.K < 1 || c.B < 1 || c.B > c.K || c.B > RAMBO_MAX_B || c.R < 1 || c.R > RAMBO_MAX_R || c.eta < 1 ||
        (uint64_t)c.R * c.eta > RAMBO_MAX_RETA || c.k < 1 || c.k > 32 || c.m < 64 || c.m > (1ull << 48) ||
        (c.flags & ~(RAMBO_FLAG_IDENTITY_PARTITION | RAMBO_FLAG_RAW_KEYS)))
        return fail(nullptr, RAMBO_EINVAL, "rambo_create: configuration out of range");

    rambo *h = new (std::nothrow) rambo();
    if (!h)
        return fail(nullptr, RAMBO_ENOMEM, "rambo_create: host allocation failed");
    h->cfg = c;
    h->S = next_pow2(c.B < 8 ? 8u : c.B);
    h->SW = h->S >= 32 ? h->S / 32 : 1;
    h->W = (c.K + 31) / 32;
    // words per repetition, rounded up to 4 so every row block is 16-byte aligned
    h->words_per_rep = div_up(div_up(c.m * h->S, 32), 4) * 4;
    h->index_bytes = (uint64_t)c.R * h->words_per_rep * 4;
    plan_partition(h);
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            h->num_cus = cus;
        (void)hipGetLastError();
    }

    // Seeds: one splitmix64 stream, in the documented order.
    uint64_t st = c.seed;
    PartitionArgs pa{};
    for (uint32_t r = 0; r < c.R; ++r) {
        pa.a[r] = 1 + splitmix64_next(st) % (kP61 - 1);
        pa.b[r] = splitmix64_next(st) % kP61;
    }
    Params &P = h->P;
    for (uint32_t r = 0; r < c.R; ++r)
        for (uint32_t j = 0; j < c.eta; ++j) {
            const uint32_t t = r * c.eta + j;
            P.seeds[t] = splitmix64_next(st) | 1u;   // odd multiplier of the multiply-shift hash
            P.rep_of[t] = (uint8_t)r;
            if (j == 0)
                P.rep_first |= 1u << t;
            if (j + 1 == c.eta)
                P.rep_last |= 1u << t;
        }
    P.m = c.m;
    P.words_per_rep = h->words_per_rep;
    P.raw_keys = (c.flags & RAMBO_FLAG_RAW_KEYS) ? 1u : 0u;
    P.kmask = c.k >= 32 || P.raw_keys ? ~0ull : ((1ull << (2 * c.k)) - 1);
    P.K = c.K;
    P.B = c.B;
    P.R = c.R;
    P.eta = c.eta;
    P.k = c.k;
    P.W = h->W;
    P.S_log2 = log2_exact(h->S);
    P.m_log2 = ((c.m & (c.m - 1)) == 0) ? log2_exact(c.m) : 0;

    int rc = RAMBO_OK;
    const uint64_t cm_words = (uint64_t)c.R * c.B * h->W;
    if (hipMalloc(&h->index, h->index_bytes) != hipSuccess || hipMalloc(&h->phi, (uint64_t)c.R * c.K * 2) != hipSuccess ||
        hipMalloc(&h->cellmask, cm_words * 4) != hipSuccess || hipMalloc(&h->err, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        g_create_error = "rambo_create: device allocation failed";
        rambo_destroy(h);
        return RAMBO_ENOMEM;
    }
    if (hipEventCreateWithFlags(&h->scratch_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        h->scratch_ev = nullptr;
        g_create_error = "rambo_create: event creation failed";
        rambo_destroy(h);
        return RAMBO_EHIP;
    }
    P.index = h->index;
    P.phi = h->phi;
    P.cellmask = h->cellmask;
    P.err = h->err;
    if ((rc = hip_check(h, hipMemset(h->index, 0, h->index_bytes), "memset index")) ||
        (rc = hip_check(h, hipMemset(h->cellmask, 0, cm_words * 4), "memset cellmask")) ||
        (rc = hip_check(h, hipMemset(h->err, 0, sizeof(int)), "memset err"))) {
        g_create_error = h->last_error;
        rambo_destroy(h);
        return rc;
    }
    const uint64_t nphi = (uint64_t)c.R * c.K;
    hipLaunchKernelGGL(k_build_partition, dim3((uint32_t)div_up(nphi, kBlock)), dim3(kBlock), 0, 0, pa, c.K, c.B,
                       c.R, (uint32_t)(c.flags & RAMBO_FLAG_IDENTITY_PARTITION), h->phi);
    const uint64_t ncm = (uint64_t)c.R * h->W;
    hipLaunchKernelGGL(k_build_cellmask, dim3((uint32_t)div_up(ncm, kBlock)), dim3(kBlock), 0, 0, h->phi, c.K, c.B,
                       c.R, h->W, h->cellmask);
    if ((rc = launch_check(h, "build tables")) || (rc = hip_check(h, hipDeviceSynchronize(), "build tables")) ||
        (rc = build_member_lists(h))) {
        g_create_error = h->last_error;
        rambo_destroy(h);
        return rc;
    }
    {
        // the no-allocation entry point's scratch on this GPU: looked up here,
        // with the handle's device current; a failure shows in that call
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            h->noalloc = noalloc_scratch(dev, &h->noalloc_error);
        else
            h->noalloc_error = "hipGetDevice failed";
        (void)hipGetLastError();
    }
    *out = h;
    return RAMBO_OK;
}

extern "C" void rambo_destroy(rambo_t *h)
{
    if (!h)
        return;
    (void)hipDeviceSynchronize();
    if (h->index)
        (void)hipFree(h->index);
    if (h->phi)
        (void)hipFree(h->phi);
    if (h->cellmask)
        (void)hipFree(h->cellmask);
    if (h->member_off)
        (void)hipFree(h->member_off);
    if (h->members)
        (void)hipFree(h->members);
    if (h->err)
        (void)hipFree(h->err);
    if (h->bin_mem)
        (void)hipFree(h->bin_mem);
    if (h->rq_mem)
        (void)hipFree(h->rq_mem);
    if (h->piece_mem)
        (void)hipFree(h->piece_mem);
    for (void *p : h->retired)
        (void)hipFree(p);
    if (h->scratch_ev)
        (void)hipEventDestroy(h->scratch_ev);
    for (hipEvent_t e : h->ev_pool)
        (void)hipEventDestroy(e);
    delete h;
}

extern "C" int rambo_set_timing(rambo_t *h, int enable)
{
    if (!h)
        return RAMBO_EINVAL;
    h->timing = enable != 0;
    return RAMBO_OK;
}

extern "C" int rambo_get_stage_times(rambo_t *h, char *names, float *ms, uint32_t *calls, int max_stages)
{
    if (!h || max_stages < 0 || (max_stages > 0 && (!names || !ms)))
        return RAMBO_EINVAL;
    constexpr int kSlot = 48;
    struct Acc {
        std::string name;
        float ms;
        uint32_t calls;
    };
    std::vector<Acc> acc;
    int rc = RAMBO_OK;
    for (const auto &s : h->stages) {
        float t = 0.f;
        if (rc == RAMBO_OK && (rc = hip_check(h, hipEventSynchronize(s.b), "rambo_get_stage_times")) == RAMBO_OK)
            rc = hip_check(h, hipEventElapsedTime(&t, s.a, s.b), "rambo_get_stage_times");
        if (rc)
            break;
        auto it = std::find_if(acc.begin(), acc.end(), [&](const Acc &e) { return e.name == s.name; });
        if (it == acc.end()) {
            acc.push_back({s.name, t, 1u});
        } else {
            it->ms += t;
            it->calls += 1;
        }
    }
    h->stages.clear();
    h->ev_used = 0;
    if (rc)
        return rc;
    const int n = (int)acc.size() < max_stages ? (int)acc.size() : max_stages;
    for (int i = 0; i < n; ++i) {
        std::memset(names + (size_t)i * kSlot, 0, kSlot);
        std::strncpy(names + (size_t)i * kSlot, acc[i].name.c_str(), kSlot - 1);
        ms[i] = acc[i].ms;
        if (calls)
            calls[i] = acc[i].calls;
    }
    return (int)acc.size();
}

extern "C" int rambo_set_query_policy(rambo_t *h, int mode, uint32_t chunk_bytes, uint32_t waves_per_cu)
{
    if (!h || mode < RAMBO_QUERY_AUTO || mode > RAMBO_QUERY_QUEUE || chunk_bytes > (1u << 24) ||
        waves_per_cu > 64)
        return RAMBO_EINVAL;
    h->query_mode = mode;
    h->query_chunk = chunk_bytes ? chunk_bytes : 512;
    h->query_waves_per_cu = waves_per_cu ? waves_per_cu : 16;
    return RAMBO_OK;
}

extern "C" int rambo_set_insert_policy(rambo_t *h, int mode, uint64_t scratch_bytes)
{
    if (!h || mode < RAMBO_INSERT_AUTO || mode > RAMBO_INSERT_PARTITIONED_WALKER)
        return RAMBO_EINVAL;
    if (scratch_bytes != h->scratch_limit && h->bin_mem) {
        const int rc = hip_check(h, hipDeviceSynchronize(), "rambo_set_insert_policy");
        if (rc)
            return rc;
        if (h->recorded_insert)
            h->retired.push_back(h->bin_mem);   // a captured insert may still replay on it
        else
            (void)hipFree(h->bin_mem);
        h->bin_mem = nullptr;
    }
    h->insert_mode = mode;
    h->scratch_limit = scratch_bytes;
    return RAMBO_OK;
}

// Release the insert scratch (kept for a captured insert that may replay).
int release_scratch(rambo *h, const char *what)
{
    if (!h->bin_mem)
        return RAMBO_OK;
    const int rc = hip_check(h, hipDeviceSynchronize(), what);
    if (rc)
        return rc;
    if (h->recorded_insert)
        h->retired.push_back(h->bin_mem);
    else
        (void)hipFree(h->bin_mem);
    h->bin_mem = nullptr;
    return RAMBO_OK;
}

extern "C" int rambo_set_insert_tiles(rambo_t *h, const rambo_insert_tiles *t)
{
    if (!h)
        return RAMBO_EINVAL;
    const rambo_insert_tiles w = t ? *t : rambo_insert_tiles{};
    if (w.steps > 2 || (w.stage_b_tile && w.stage_b_tile != 8192 && w.stage_b_tile != 16384 &&
                        w.stage_b_tile != 32768) ||
        (w.groups && w.groups != 1 && w.groups != 2 && w.groups != 4 && w.groups != 8) ||
        (w.fine_bits && (w.fine_bits < 8 || w.fine_bits > 12)))
        return fail(h, RAMBO_EINVAL, "rambo_set_insert_tiles: value out of range");
    const rambo_insert_tiles old = h->tiles;
    if (std::memcmp(&old, &w, sizeof w) == 0)
        return RAMBO_OK;
    // the scratch is laid out for the old shapes: release it before the
    // partition geometry changes
    if (const int rc = release_scratch(h, "rambo_set_insert_tiles"))
        return rc;
    h->tiles = w;
    plan_partition(h);
    if (w.fine_bits && !h->part_ok) {
        h->tiles = old;
        plan_partition(h);
        return fail(h, RAMBO_EINVAL, "rambo_set_insert_tiles: fine_bits leaves too many coarse buckets");
    }
    return RAMBO_OK;
}

extern "C" int rambo_get_insert_tiles(rambo_t *h, rambo_insert_tiles *out)
{
    if (!h || !out)
        return RAMBO_EINVAL;
    const BinGeom &G = h->bin;
    const StageAPieces AP = stage_a_pieces(h);
    out->steps = AP.fn ? AP.steps : 0u;
    out->stage_b_tile = stage_b(G, h->tiles.stage_b_tile).tile;
    out->groups = h->bin_mem && G.ncb ? (G.na + G.ncb - 1) / G.ncb : h->tiles.groups;
    out->fine_bits = G.fb;
    return RAMBO_OK;
}

// Alg. 1 with one atomic OR per bit target, straight into the index.
int insert_seqs_direct(rambo *h, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_seqs,
                       const uint8_t *chars, uint64_t n_chars, hipStream_t stream)
{
    note_insert(h, stream);
    const uint64_t waves = div_up(n_chars, kChunk);
    const InsertSeqsFn ins = pick_shape<InsertSeqsFn, InsertSeqsK>(h->cfg.R, h->cfg.eta);
    StageScope sc(h, "k_insert_seqs", stream);
    hipLaunchKernelGGL(ins, dim3((uint32_t)div_up(waves, kWavesPerBlock)), dim3(kBlock), 0, stream, h->P, set_ids,
                       offsets, n_seqs, chars, n_chars, kChunk);
    return launch_check(h, "rambo_insert_seqs");
}

// Sequence input needs k-mer terms: a raw-key index refuses it.
int refuse_raw_keys(rambo *h, const char *what)
{
    if (!(h->cfg.flags & RAMBO_FLAG_RAW_KEYS))
        return RAMBO_OK;
    return fail(h, RAMBO_EINVAL, std::string(what) + ": the index holds raw 64-bit keys, not k-mers");
}

extern "C" int rambo_insert_kmers(rambo_t *h, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_sets,
                                  const uint64_t *codes, uint64_t n_codes, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (n_sets == 0 || n_codes == 0)
        return RAMBO_OK;
    if (!set_ids || !offsets || !codes)
        return fail(h, RAMBO_EINVAL, "rambo_insert_kmers: NULL array");
    if (use_partitioned(h, n_codes)) {
        ScratchUse su(h, stream);
        return insert_kmers_partitioned(h, set_ids, offsets, n_sets, codes, n_codes, stream);
    }
    note_insert(h, stream);
    StageScope sc(h, "k_insert_kmers", stream);
    hipLaunchKernelGGL(k_insert_kmers, dim3((uint32_t)div_up(n_codes, kBlock)), dim3(kBlock), 0, stream, h->P,
                       set_ids, offsets, n_sets, codes, n_codes);
    return launch_check(h, "rambo_insert_kmers");
}

extern "C" int rambo_insert_seqs(rambo_t *h, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_seqs,
                                 const uint8_t *chars, uint64_t n_chars, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (const int rr = refuse_raw_keys(h, "rambo_insert_seqs"))
        return rr;
    if (n_seqs == 0 || n_chars == 0)
        return RAMBO_OK;
    if (!set_ids || !offsets || !chars)
        return fail(h, RAMBO_EINVAL, "rambo_insert_seqs: NULL array");
    if (use_partitioned(h, n_chars)) {
        ScratchUse su(h, stream);
        return insert_seqs_partitioned(h, set_ids, offsets, n_seqs, chars, n_chars, stream);
    }
    return insert_seqs_direct(h, set_ids, offsets, n_seqs, chars, n_chars, stream);
}

extern "C" int rambo_query_kmers(rambo_t *h, const uint64_t *codes, uint64_t n, uint32_t *out_masks,
                                 hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (n == 0)
        return RAMBO_OK;
    if (!codes || !out_masks)
        return fail(h, RAMBO_EINVAL, "rambo_query_kmers: NULL array");
    with_row_words(h, QueryKmersLaunch{h, codes, n, out_masks, stream});
    return launch_check(h, "rambo_query_kmers");
}

extern "C" int rambo_query_termsets(rambo_t *h, const uint64_t *offsets, uint64_t n_sets, const uint64_t *codes,
                                    uint64_t n_codes, uint32_t *out_masks, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (n_sets == 0)
        return RAMBO_OK;
    if (!offsets || !out_masks || (n_codes > 0 && !codes))
        return fail(h, RAMBO_EINVAL, "rambo_query_termsets: NULL array");
    with_row_words(h, QueryTermsetsLaunch{h, offsets, n_sets, codes, n_codes, out_masks, stream});
    return launch_check(h, "rambo_query_termsets");
}

extern "C" int rambo_query_seqs(rambo_t *h, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars,
                                uint64_t n_chars, uint32_t *out_masks, uint32_t *out_nkmers, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (const int rr = refuse_raw_keys(h, "rambo_query_seqs"))
        return rr;
    if (n_reads == 0)
        return RAMBO_OK;
    if (!offsets || !out_masks || (n_chars > 0 && !chars))
        return fail(h, RAMBO_EINVAL, "rambo_query_seqs: NULL array");
    if (wave_per_read(h, n_reads, n_chars)) {
        with_row_words(h, QuerySeqsLaunch{h, offsets, n_reads, chars, n_chars, out_masks, out_nkmers, stream, h->rq});
        return launch_check(h, "rambo_query_seqs");
    }
    ScratchUse su(h, stream);
    int rc = ensure_read_queue(h, n_reads);
    if (rc)
        return rc;
    if (capturing(stream))
        h->rq_recorded = true;
    launch_read_queue(h, h->rq, offsets, n_reads, nullptr, n_reads, chars, n_chars, out_masks, out_nkmers, stream);
    return launch_check(h, "rambo_query_seqs");
}

// Alg. 2 with Sec. 3.2.1 per read, then the answers as ID lists, with the
// per-read state in rq and the scan's tile totals in scan_part (both hold
// n_reads reads).
int query_seqs_ids_on(rambo *h, const ReadQueue &rq, uint64_t *scan_part, const uint64_t *offsets,
                      uint64_t n_reads, const uint8_t *chars, uint64_t n_chars, uint64_t *id_offsets, uint32_t *ids,
                      uint64_t cap, uint32_t *out_nkmers, hipStream_t stream, const char *what)
{
    // group masks and window counts only: the answers stay in the per-read state
    if (wave_per_read(h, n_reads, n_chars))
        with_row_words(h, QuerySeqsLaunch{h, offsets, n_reads, chars, n_chars, nullptr, out_nkmers, stream, rq});
    else
        launch_read_queue(h, rq, offsets, n_reads, nullptr, n_reads, chars, n_chars, nullptr, out_nkmers, stream);
    const uint64_t waves = std::min<uint64_t>(div_up(n_reads, kWave), (uint64_t)h->num_cus * 32);
    const dim3 grid((uint32_t)div_up(waves, kWavesPerBlock));
    const size_t lds = (size_t)kWavesPerBlock * h->cfg.R * h->SW * 4;
    {
        StageScope sc(h, "k_ids_count", stream);
        hipLaunchKernelGGL(k_ids_count, grid, dim3(kBlock), lds + (size_t)kWavesPerBlock * kSortCap * 4, stream, h->P,
                           rq, n_reads, h->SW, id_offsets);
    }
    const uint64_t nb = div_up(n_reads, kScanTile);
    {
        StageScope sc(h, "k_scan64", stream);
        hipLaunchKernelGGL(k_scan64_tiles, dim3((uint32_t)nb), dim3(256), 0, stream, id_offsets, n_reads, id_offsets,
                           scan_part);
        hipLaunchKernelGGL(k_scan64_part, dim3(1), dim3(1024), 0, stream, scan_part, nb, id_offsets, n_reads, cap,
                           h->err);
        hipLaunchKernelGGL(k_scan64_add, dim3((uint32_t)div_up(n_reads, 256)), dim3(256), 0, stream, id_offsets,
                           n_reads, scan_part);
    }
    {
        StageScope sc(h, "k_ids_write", stream);
        hipLaunchKernelGGL(k_ids_write, grid, dim3(kBlock), lds + (size_t)kWavesPerBlock * kSortCap * 4, stream, h->P,
                           rq, n_reads, h->SW, id_offsets, ids, cap);
    }
    return launch_check(h, what);
}

int query_seqs_ids_args(rambo *h, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars, uint64_t n_chars,
                        const uint64_t *id_offsets, const uint32_t *ids, uint64_t cap, const char *what)
{
    if (const int rr = refuse_raw_keys(h, what))
        return rr;
    if (!id_offsets || (n_reads > 0 && !offsets) || (n_chars > 0 && !chars) || (cap > 0 && !ids))
        return fail(h, RAMBO_EINVAL, std::string(what) + ": NULL array");
    return RAMBO_OK;
}

// id_offsets[0] = 0 for an empty batch, by a fill kernel (no memset node if
// recorded into a graph).
int query_seqs_ids_empty(rambo *h, uint64_t *id_offsets, hipStream_t stream, const char *what)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlock), 0, stream, reinterpret_cast<uint32_t *>(id_offsets),
                       (uint64_t)2, 0u);
    return launch_check(h, what);
}

extern "C" int rambo_query_seqs_ids(rambo_t *h, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars,
                                    uint64_t n_chars, uint64_t *id_offsets, uint32_t *ids, uint64_t cap,
                                    uint32_t *out_nkmers, hipStream_t stream)
{
    static const char *what = "rambo_query_seqs_ids";
    if (!h)
        return RAMBO_EINVAL;
    if (const int rc = query_seqs_ids_args(h, offsets, n_reads, chars, n_chars, id_offsets, ids, cap, what))
        return rc;
    if (n_reads == 0)
        return query_seqs_ids_empty(h, id_offsets, stream, what);
    ScratchUse su(h, stream);
    int rc = ensure_read_queue(h, n_reads);
    if (rc)
        return rc;
    if (capturing(stream))
        h->rq_recorded = true;
    return query_seqs_ids_on(h, h->rq, h->scan_part, offsets, n_reads, chars, n_chars, id_offsets, ids, cap,
                             out_nkmers, stream, what);
}

// ------------------------------------- ID lists without allocating memory

// The per-read state and scan totals of rambo_query_seqs_ids_noalloc: one
// array per GPU for the life of the process, shared by every handle and
// call on that GPU.
namespace {

static __device__ __align__(256) uint8_t scratch[RAMBO_NOALLOC_SCRATCH_BYTES];

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// The device address of this GPU's copy of `scratch` (the array's name is
// only a host-side stand-in), looked up once per device with that device
// current; nullptr, with the reason in *err, if the lookup fails.
void *noalloc_scratch(int dev, std::string *err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        *err = "device ordinal out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_noalloc_ptr[dev] = ptr;
    }
    return g_noalloc_ptr[dev];
}

// Bytes of the per-read state (rounded to 256) plus the scan's tile totals
// for n reads.
uint64_t noalloc_bytes(const rambo *h, uint64_t n)
{
    return div_up(read_queue_bytes(h, n), 256) * 256 + 8 * (div_up(n, kScanTile) + 1);
}

}  // namespace

extern "C" uint64_t rambo_query_seqs_ids_noalloc_max_reads(const rambo_t *h)
{
    if (!h)
        return 0;
    uint64_t lo = 0, hi = RAMBO_NOALLOC_SCRATCH_BYTES;   // noalloc_bytes(h, lo) fits
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        (noalloc_bytes(h, mid) <= RAMBO_NOALLOC_SCRATCH_BYTES ? lo : hi) = mid;
        if (lo != mid)
            hi = mid - 1;
    }
    return lo;
}

extern "C" int rambo_query_seqs_ids_noalloc(rambo_t *h, const uint64_t *offsets, uint64_t n_reads,
                                            const uint8_t *chars, uint64_t n_chars, uint64_t *id_offsets,
                                            uint32_t *ids, uint64_t cap, uint32_t *out_nkmers, hipStream_t stream)
{
    static const char *what = "rambo_query_seqs_ids_noalloc";
    if (!h)
        return RAMBO_EINVAL;
    if (const int rc = query_seqs_ids_args(h, offsets, n_reads, chars, n_chars, id_offsets, ids, cap, what))
        return rc;
    if (!h->noalloc)
        return fail(h, RAMBO_EHIP, std::string(what) + ": no scratch on this GPU (" + h->noalloc_error + ")");
    if (n_reads == 0)
        return query_seqs_ids_empty(h, id_offsets, stream, what);
    if (noalloc_bytes(h, n_reads) > RAMBO_NOALLOC_SCRATCH_BYTES)
        return fail(h, RAMBO_EINVAL, std::string(what) + ": " + std::to_string(n_reads) + " reads need " +
                                         std::to_string(noalloc_bytes(h, n_reads)) + " bytes of scratch, more than " +
                                         std::to_string((uint64_t)RAMBO_NOALLOC_SCRATCH_BYTES));
    uint8_t *base = static_cast<uint8_t *>(h->noalloc);
    const ReadQueue rq = carve_read_queue(h, base, n_reads);
    uint64_t *scan_part = reinterpret_cast<uint64_t *>(base + div_up(read_queue_bytes(h, n_reads), 256) * 256);
    return query_seqs_ids_on(h, rq, scan_part, offsets, n_reads, chars, n_chars, id_offsets, ids, cap, out_nkmers,
                             stream, what);
}

extern "C" int rambo_fill_counts(rambo_t *h, uint64_t *out, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (!out)
        return fail(h, RAMBO_EINVAL, "rambo_fill_counts: NULL array");
    const uint64_t n = (uint64_t)h->cfg.R * h->cfg.B;
    hipLaunchKernelGGL(k_zero_u32, dim3((uint32_t)div_up(2 * n, kBlock)), dim3(kBlock), 0, stream,
                       reinterpret_cast<uint32_t *>(out), 2 * n);
    StageScope sc(h, "k_fill_counts", stream);
    hipLaunchKernelGGL(k_fill_counts, dim3((uint32_t)div_up(h->words_per_rep, kFillTile), h->cfg.R), dim3(kBlock),
                       (size_t)h->S * 4, stream, h->index, h->words_per_rep, h->S, h->cfg.B,
                       reinterpret_cast<unsigned long long *>(out));
    return launch_check(h, "rambo_fill_counts");
}

extern "C" int rambo_extract_kmers(rambo_t *h, const uint64_t *offsets, uint64_t n_seqs, const uint8_t *chars,
                                   uint64_t n_chars, uint64_t *out_codes, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (const int rr = refuse_raw_keys(h, "rambo_extract_kmers"))
        return rr;
    if (n_chars == 0)
        return RAMBO_OK;
    if (!chars || !out_codes || (n_seqs > 0 && !offsets))
        return fail(h, RAMBO_EINVAL, "rambo_extract_kmers: NULL array");
    if (n_seqs == 0) {
        // no sequence holds any byte: every entry is "no window" (a fill
        // kernel, so that a recorded call holds no memset node)
        hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)std::min<uint64_t>(div_up(2 * n_chars, kBlock), 4096)),
                           dim3(kBlock), 0, stream, reinterpret_cast<uint32_t *>(out_codes), 2 * n_chars, ~0u);
        return launch_check(h, "rambo_extract_kmers");
    }
    const uint64_t waves = div_up(n_chars, kChunk);
    StageScope sc(h, "k_extract", stream);
    hipLaunchKernelGGL(k_extract, dim3((uint32_t)div_up(waves, kWavesPerBlock)), dim3(kBlock), 0, stream, h->cfg.k,
                       h->P.kmask, offsets, n_seqs, chars, n_chars, kChunk, out_codes);
    return launch_check(h, "rambo_extract_kmers");
}

extern "C" int rambo_query_kmers_plain(rambo_t *h, const uint64_t *codes, uint64_t n, uint32_t *out_masks,
                                       hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (n == 0)
        return RAMBO_OK;
    if (!codes || !out_masks)
        return fail(h, RAMBO_EINVAL, "rambo_query_kmers_plain: NULL array");
    for (uint64_t q = 0; q < n; ++q)
        with_row_words(h, QueryKmersLaunch{h, codes + q, 1, out_masks + q * h->W, stream});
    return launch_check(h, "rambo_query_kmers_plain");
}

extern "C" int rambo_query_seqs_plain(rambo_t *h, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars,
                                      uint64_t n_chars, uint32_t *out_masks, uint32_t *out_nkmers,
                                      hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (const int rr = refuse_raw_keys(h, "rambo_query_seqs_plain"))
        return rr;
    if (n_reads == 0)
        return RAMBO_OK;
    if (!offsets || !out_masks || (n_chars > 0 && !chars))
        return fail(h, RAMBO_EINVAL, "rambo_query_seqs_plain: NULL array");
    for (uint64_t q = 0; q < n_reads; ++q)
        with_row_words(h, QuerySeqsLaunch{h, offsets + q, 1, chars, n_chars, out_masks + q * h->W,
                                          out_nkmers ? out_nkmers + q : nullptr, stream, h->rq});
    return launch_check(h, "rambo_query_seqs_plain");
}

extern "C" int rambo_fold(rambo_t *h, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    const rambo_config c = h->cfg;
    if (c.B < 2 || c.B % 2 != 0)
        return fail(h, RAMBO_EINVAL, "rambo_fold: B must be even");
    if (h->servers)
        return fail(h, RAMBO_EINVAL, "rambo_fold: a query server is attached to the handle");
    const uint32_t half = c.B / 2;
    const uint32_t S2 = next_pow2(half < 8 ? 8u : half);
    const uint64_t wpr2 = div_up(div_up(c.m * S2, 32), 4) * 4;
    uint32_t *index2 = nullptr;
    if (hipMalloc(&index2, (uint64_t)c.R * wpr2 * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, RAMBO_ENOMEM, "rambo_fold: device allocation failed");
    }
    const uint64_t n2 = (uint64_t)c.R * wpr2;
    {
        StageScope sc(h, "k_fold", stream);
        if (S2 == 32 && h->S == 64)
            hipLaunchKernelGGL(k_fold_narrow<1>, dim3((uint32_t)div_up(n2 / 4, kBlock)), dim3(kBlock), 0, stream,
                               h->index, index2, c.R, c.m, h->words_per_rep, wpr2, half);
        else if (S2 == 64 && h->S == 128)
            hipLaunchKernelGGL(k_fold_narrow<2>, dim3((uint32_t)div_up(n2 / 4, kBlock)), dim3(kBlock), 0, stream,
                               h->index, index2, c.R, c.m, h->words_per_rep, wpr2, half);
        else
            hipLaunchKernelGGL(k_fold, dim3((uint32_t)div_up(n2, kBlock)), dim3(kBlock), 0, stream, h->index, index2,
                               c.R, c.m, h->S, S2, h->words_per_rep, wpr2, half);
    }
    const uint64_t nphi = (uint64_t)c.R * c.K;
    hipLaunchKernelGGL(k_phi_mod, dim3((uint32_t)div_up(nphi, kBlock)), dim3(kBlock), 0, stream, h->phi, nphi, half);
    int rc = launch_check(h, "rambo_fold");
    if (!rc)
        rc = hip_check(h, hipStreamSynchronize(stream), "rambo_fold");
    if (rc) {
        (void)hipFree(index2);
        return rc;
    }
    // the handle now describes the folded index; tables and scratch whose
    // shape depends on B are rebuilt or dropped
    (void)hipFree(h->index);
    h->index = index2;
    h->cfg.B = half;
    h->S = S2;
    h->SW = S2 >= 32 ? S2 / 32 : 1;
    h->words_per_rep = wpr2;
    h->index_bytes = (uint64_t)c.R * wpr2 * 4;
    Params &P = h->P;
    P.index = index2;
    P.B = half;
    P.S_log2 = log2_exact(S2);
    P.words_per_rep = wpr2;
    if (h->bin_mem) {
        (void)hipFree(h->bin_mem);
        h->bin_mem = nullptr;
    }
    plan_partition(h);
    if (h->rq_mem) {
        (void)hipFree(h->rq_mem);
        h->rq_mem = nullptr;
        h->rq_cap = 0;
    }
    return rebuild_tables(h);
}

// ------------------------------------------------------------ save / load

namespace {

constexpr char kFileMagic[8] = {'R', 'A', 'M', 'B', 'O', 'I', 'X', '1'};

struct FileHeader {
    char magic[8];
    rambo_config cfg;
    uint64_t words_per_rep;
    uint64_t index_bytes;
    uint32_t row_bits;
    uint32_t reserved;
};

// Copy n bytes between the device and a file through a pinned bounce buffer.
int stream_file(rambo *h, FILE *f, void *dev, uint64_t n, bool to_file)
{
    constexpr uint64_t kChunk = 64ull << 20;
    void *buf = nullptr;
    if (hipHostMalloc(&buf, std::min(n, kChunk) + 1, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, RAMBO_ENOMEM, "save/load: pinned buffer");
    }
    int rc = RAMBO_OK;
    for (uint64_t o = 0; o < n && !rc; o += kChunk) {
        const uint64_t len = std::min(kChunk, n - o);
        uint8_t *d = static_cast<uint8_t *>(dev) + o;
        if (to_file) {
            rc = hip_check(h, hipMemcpy(buf, d, len, hipMemcpyDeviceToHost), "rambo_save");
            if (!rc && std::fwrite(buf, 1, len, f) != len)
                rc = fail(h, RAMBO_EIO, "rambo_save: write failed");
        } else {
            if (std::fread(buf, 1, len, f) != len)
                rc = fail(h, RAMBO_EIO, "rambo_load: file too short");
            else
                rc = hip_check(h, hipMemcpy(d, buf, len, hipMemcpyHostToDevice), "rambo_load");
        }
    }
    (void)hipHostFree(buf);
    return rc;
}

}  // namespace

extern "C" int rambo_save(rambo_t *h, const char *path, hipStream_t stream)
{
    if (!h || !path)
        return RAMBO_EINVAL;
    int rc = hip_check(h, hipStreamSynchronize(stream), "rambo_save");
    if (rc)
        return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return fail(h, RAMBO_EIO, std::string("rambo_save: cannot open ") + path);
    FileHeader hd{};
    std::memcpy(hd.magic, kFileMagic, 8);
    hd.cfg = h->cfg;
    hd.words_per_rep = h->words_per_rep;
    hd.index_bytes = h->index_bytes;
    hd.row_bits = h->S;
    if (std::fwrite(&hd, sizeof hd, 1, f) != 1)
        rc = fail(h, RAMBO_EIO, "rambo_save: write failed");
    if (!rc)
        rc = stream_file(h, f, h->phi, (uint64_t)h->cfg.R * h->cfg.K * 2, true);
    if (!rc)
        rc = stream_file(h, f, h->index, h->index_bytes, true);
    if (std::fclose(f) != 0 && !rc)
        rc = fail(h, RAMBO_EIO, "rambo_save: close failed");
    return rc;
}

extern "C" int rambo_load(const char *path, rambo_t **out)
{
    if (!path || !out)
        return fail(nullptr, RAMBO_EINVAL, "rambo_load: NULL argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return fail(nullptr, RAMBO_EIO, std::string("rambo_load: cannot open ") + path);
    FileHeader hd{};
    if (std::fread(&hd, sizeof hd, 1, f) != 1 || std::memcmp(hd.magic, kFileMagic, 8) != 0) {
        std::fclose(f);
        return fail(nullptr, RAMBO_EINVAL, "rambo_load: not a RAMBO index file");
    }
    rambo_t *h = nullptr;
    int rc = rambo_create(&hd.cfg, &h);
    if (rc) {
        std::fclose(f);
        return rc;
    }
    if (hd.words_per_rep != h->words_per_rep || hd.index_bytes != h->index_bytes || hd.row_bits != h->S) {
        std::fclose(f);
        rambo_destroy(h);
        return fail(nullptr, RAMBO_EINVAL, "rambo_load: layout does not match the configuration");
    }
    rc = stream_file(h, f, h->phi, (uint64_t)hd.cfg.R * hd.cfg.K * 2, false);
    if (!rc) {
        // the partition as saved (it may differ from the one the seed gives,
        // e.g. after folding); it must stay within the cells
        std::vector<uint16_t> phi((size_t)hd.cfg.R * hd.cfg.K);
        rc = hip_check(h, hipMemcpy(phi.data(), h->phi, phi.size() * 2, hipMemcpyDeviceToHost), "rambo_load");
        for (size_t i = 0; !rc && i < phi.size(); ++i)
            if (phi[i] >= hd.cfg.B)
                rc = fail(h, RAMBO_EINVAL, "rambo_load: partition value out of range");
    }
    if (!rc)
        rc = stream_file(h, f, h->index, h->index_bytes, false);
    std::fclose(f);
    if (!rc)
        rc = rebuild_tables(h);
    if (rc) {
        g_create_error = h->last_error;
        rambo_destroy(h);
        return rc;
    }
    h->index_zero = false;
    *out = h;
    return RAMBO_OK;
}

extern "C" int rambo_get_config(const rambo_t *h, rambo_config *out)
{
    if (!h || !out)
        return RAMBO_EINVAL;
    *out = h->cfg;
    return RAMBO_OK;
}

extern "C" int rambo_clear(rambo_t *h, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    if (capturing(stream)) {
        // a fill kernel, not a memset node, in a graph; the host does not
        // learn that the index is zero (the graph runs later)
        hipLaunchKernelGGL(k_zero_u32, dim3(4096), dim3(kBlock), 0, stream, h->index, h->index_bytes / 4);
        return launch_check(h, "rambo_clear");
    }
    const int rc = hip_check(h, hipMemsetAsync(h->index, 0, h->index_bytes, stream), "rambo_clear");
    if (rc == RAMBO_OK)
        h->index_zero = true;
    return rc;
}

extern "C" int rambo_get_info(const rambo_t *h, rambo_info *out)
{
    if (!h || !out)
        return RAMBO_EINVAL;
    out->row_bits = h->S;
    out->mask_words = h->W;
    out->words_per_rep = h->words_per_rep;
    out->index_bytes = h->index_bytes;
    out->index = h->index;
    return RAMBO_OK;
}

extern "C" int rambo_copy_index(rambo_t *h, uint64_t word_offset, uint64_t n_words, void *dst, hipStream_t stream)
{
    if (!h || (n_words && !dst))
        return RAMBO_EINVAL;
    const uint64_t total = h->index_bytes / 4;
    if (word_offset > total || n_words > total - word_offset)
        return fail(h, RAMBO_EINVAL, "rambo_copy_index: range outside the index");
    if (n_words == 0)
        return RAMBO_OK;
    return hip_check(h, hipMemcpyAsync(dst, h->index + word_offset, n_words * 4, hipMemcpyDefault, stream),
                     "rambo_copy_index");
}

extern "C" int rambo_get_partition(rambo_t *h, uint32_t *out)
{
    if (!h || !out)
        return RAMBO_EINVAL;
    const uint64_t n = (uint64_t)h->cfg.R * h->cfg.K;
    uint16_t *tmp = new (std::nothrow) uint16_t[n];
    if (!tmp)
        return fail(h, RAMBO_ENOMEM, "rambo_get_partition: host allocation failed");
    const int rc = hip_check(h, hipMemcpy(tmp, h->phi, n * 2, hipMemcpyDeviceToHost), "rambo_get_partition");
    if (rc == RAMBO_OK)
        for (uint64_t i = 0; i < n; ++i)
            out[i] = tmp[i];
    delete[] tmp;
    return rc;
}

extern "C" int rambo_sync_status(rambo_t *h, hipStream_t stream)
{
    if (!h)
        return RAMBO_EINVAL;
    int rc = hip_check(h, hipStreamSynchronize(stream), "rambo_sync_status");
    if (rc)
        return rc;
    int e = 0;
    if ((rc = hip_check(h, hipMemcpy(&e, h->err, sizeof(int), hipMemcpyDeviceToHost), "rambo_sync_status")))
        return rc;
    if (e && (rc = hip_check(h, hipMemset(h->err, 0, sizeof(int)), "rambo_sync_status")))
        return rc;
    if (e & kErrSetId)
        return fail(h, RAMBO_ERANGE, "a set id >= K was seen on the device");
    if (e & kErrCode)
        return fail(h, RAMBO_ECODE, "a k-mer code >= 4^k was seen on the device");
    if (e & kErrOverflow)
        return fail(h, RAMBO_EOVERFLOW, "an answer list did not fit the capacity given");
    return RAMBO_OK;
}

extern "C" const char *rambo_last_error(const rambo_t *h)
{
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

#include "serve.hpp"
