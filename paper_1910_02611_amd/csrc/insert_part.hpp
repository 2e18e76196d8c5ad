// Partitioned bulk insertion (Alg. 1 without global atomics).
//
// A random atomicOr per bit target is bound by the device's atomic rate, and
// a scattered 4-byte store per target by the L2's request rate, not by HBM
// bandwidth.  For bulk inserts the targets are instead partitioned by
// address, twice, and applied region by region in LDS:
//
//  A  k_bin_windows : a workgroup takes the R*eta targets (global bit
//                     addresses of the bit-sliced index) of a tile of windows,
//                     counting-sorts them in LDS by coarse bucket, reserves one
//                     run per bucket in the bucket's slab (one atomicAdd per
//                     bucket and tile) and writes each run with coalesced
//                     stores.
//  B  k_bin_regions : each tile of a coarse bucket's slab is split the same
//                     way into the bucket's fine buckets (index regions of
//                     2^rb bits).
// Stages A and B keep a tile's targets in registers while they are counted:
// the counting atomic returns each target's rank inside its bucket, so after
// the scan every target goes straight to its slot in the sorted LDS tile.
//  C  k_apply_regions: one workgroup per region loads the region into LDS,
//                     ORs in its targets with LDS atomics and writes it back.
//
// OR is order-free and idempotent, so the order in which runs are filled does
// not change the index.  A run that does not fit in its slab is applied with
// global atomics instead, so every input is inserted whatever its skew.
#pragma once

#include "kernels.hpp"

namespace rambo_dev {

constexpr uint32_t kRegionLog2Max = 20;         // regions of at most 2^20 bits (128 KiB of LDS)
constexpr int kBlockC = 1024;                   // workgroup of stage C (one per CU: its region fills most of the LDS)
constexpr uint32_t kXcds = 8;                   // accelerator complex dies: workgroups are dealt to them in turn
constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr uint32_t kFail = 0xFFFFFFFFu;
constexpr uint16_t kNoBucket = 0xFFFFu;
constexpr int kBlockP = 512;                    // workgroup of stages A and B
constexpr int kWavesP = kBlockP / kWave;
constexpr uint32_t kTileA = 8192;               // targets per round in stage A
constexpr uint32_t kTileB = 8192;               // slab entries per tile in stage B
constexpr uint32_t kMaxTargetsPerWindow = kTileA / kBlockP;   // R*eta the partitioned path supports

// Slab A holds na * nwg chunks of capA entries: chunk (b, g) at
// slabA + (b * nwg + g) * capA, filled by producer g with entries of coarse
// bucket b; fillA[b * nwg + g] counts them.  The stage-A kernels that
// reserve runs with global atomics use one chunk per bucket (nwg = 1).
struct BinGeom {
    uint32_t rb;          // log2 of the bits in one region
    uint32_t fb;          // log2 of the regions in one coarse bucket
    uint32_t na;          // coarse buckets
    uint32_t nf;          // regions per coarse bucket (1 << fb)
    uint32_t nwg;         // chunks per coarse bucket (stage-A producers)
    uint64_t capA;        // slab entries per chunk
    uint64_t capB;        // slab entries per region
    uint32_t *slabA;      // na * nwg * capA
    uint32_t *fillA;      // na * nwg
    uint32_t *slabB;      // capB per region of one group of coarse buckets (at most
    uint32_t *fillB;      //   ncb * nf regions, fewer where the index ends)
    uint32_t *dirty;      // na * nf: a fallback atomic wrote into this region
    uint64_t total_words; // words of the index (all repetitions)
    uint32_t c0;          // stages B and C take the coarse buckets c0 .. c0 + ncb - 1;
    uint32_t ncb;         //   slab B and fillB hold just their regions
};

__host__ __device__ constexpr size_t lds_bytes_stage_a(uint32_t na) { return kTileA * 12ull + na * 12ull + 64; }
__host__ __device__ constexpr size_t lds_bytes_stage_b(uint32_t nf) { return kTileB * 4ull + nf * 8ull; }   // the smallest stage-B tile

// A target whose run did not fit its slab is set with a global atomic right
// away; its region is marked so that stage C reads the region back even into
// an index known to have been all zero.
__device__ __forceinline__ void fallback_or(const Params &P, const BinGeom &G, uint64_t gb)
{
    direct_or(P, gb);
    G.dirty[gb >> G.rb] = 1u;
}

// Exclusive prefix sum of cnt[0..n) into start[0..n) by the whole
// workgroup of BLK threads; returns the total.  wsum holds BLK / 64 words
// of LDS.
template <int BLK = kBlockP>
__device__ __forceinline__ uint32_t block_exclusive_scan(const uint32_t *cnt, uint32_t *start, uint32_t n,
                                                         uint32_t *wsum)
{
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t per = (n + BLK - 1) / BLK;
    const uint32_t b0 = min(threadIdx.x * per, n), b1 = min(b0 + per, n);
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b)
        s += cnt[b];
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, kWave);
        if ((int)lane >= off)
            incl += t;
    }
    if (lane == kWave - 1)
        wsum[wv] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < BLK / kWave; ++w) {
        const uint32_t ws = wsum[w];
        wbase += (uint32_t)w < wv ? ws : 0u;
        total += ws;
    }
    uint32_t run = wbase + incl - s;
    for (uint32_t b = b0; b < b1; ++b) {
        start[b] = run;
        run += cnt[b];
    }
    __syncthreads();
    return total;
}

// Reserving one run per bucket takes a global atomicAdd round trip.  The
// reservation is split so that the LDS scatter runs while the atomics are in
// flight: issue() starts them (cnt[b] entries for bucket b, at most kSlots
// buckets per thread) and resets cnt[b] to 0; finish() stores gbase[b], the
// run's first slab entry, or kFail for a run that does not fit - whose slab
// tail, if it starts inside the slab, is filled with sentinels so readers
// skip it.
constexpr uint32_t kMaxBucketsPerThread = 8;   // 4096 buckets / 512 threads

template <uint32_t kSlots, int BLK = kBlockP>
struct RunReservationT {
    uint32_t pos[kSlots];
    uint32_t c[kSlots];

    __device__ __forceinline__ void issue(uint32_t *cnt, uint32_t nb, uint32_t *fill)
    {
#pragma unroll
        for (uint32_t i = 0; i < kSlots; ++i) {
            const uint32_t b = threadIdx.x + i * BLK;
            c[i] = 0;
            pos[i] = 0;
            if (b < nb) {
                c[i] = cnt[b];
                cnt[b] = 0;
                if (c[i])
                    pos[i] = atomicAdd(fill + b, c[i]);
            }
        }
    }

    __device__ __forceinline__ void finish(uint32_t *gbase, uint32_t nb, uint32_t *slab, uint64_t cap)
    {
#pragma unroll
        for (uint32_t i = 0; i < kSlots; ++i) {
            const uint32_t b = threadIdx.x + i * BLK;
            if (b >= nb)
                continue;
            if (c[i] == 0) {
                gbase[b] = kFail;
            } else if ((uint64_t)pos[i] + c[i] <= cap) {
                gbase[b] = pos[i];
            } else {
                gbase[b] = kFail;
                for (uint64_t e = pos[i]; e < cap; ++e)
                    slab[(uint64_t)b * cap + e] = kSentinel;
            }
        }
    }
};
using RunReservation = RunReservationT<kMaxBucketsPerThread>;

// Stage A over the terms [p_begin, p_end) of a walker (WindowWalker over
// sequence windows, CodeWalker over codes or keys; init_walker(w, first,
// end) starts it).  Wave w of block g walks `rounds * steps * 64`
// consecutive terms; each round the workgroup gathers the targets of `steps`
// steps of every wave (at most kTileA), sorts them by coarse bucket in LDS
// and writes them out run by run.
template <int R_T, int ETA_T, class Walker, class Init>
__device__ __forceinline__ void bin_generic(const Params &P, const BinGeom &G, const uint32_t *set_ids,
                                            uint64_t p_begin, uint64_t p_end, uint32_t steps, uint32_t rounds,
                                            Init &&init_walker)
{
    extern __shared__ uint32_t lds[];
    uint32_t *ent = lds;                                          // kTileA: low bits of each target
    uint32_t *srt = ent + kTileA;                                 // kTileA: the same, sorted by bucket
    uint16_t *bkt = reinterpret_cast<uint16_t *>(srt + kTileA);   // kTileA: bucket of each target
    uint16_t *sbk = bkt + kTileA;                                 // kTileA: bucket, sorted
    uint32_t *cnt = reinterpret_cast<uint32_t *>(sbk + kTileA);   // na: counts, then run cursors
    uint32_t *lbase = cnt + G.na;                                 // na: first sorted slot of each bucket
    uint32_t *gbase = lbase + G.na;                               // na: first slab entry of each run
    uint32_t *wsum = gbase + G.na;                                // kWavesP
    const uint32_t shA = G.rb + G.fb;
    const uint64_t maskA = (1ull << shA) - 1;
    const uint32_t RE = P.R * P.eta;
    const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
    const uint64_t span = (uint64_t)rounds * steps * kWave;
    const uint64_t w0 = p_begin + ((uint64_t)blockIdx.x * kWavesP + wv) * span;
    const uint64_t w1 = min(w0 + span, p_end);
    const bool busy = w0 < p_end;
    Walker walker;
    if (busy)
        init_walker(walker, w0, w1);
    SetCache cache;
    cache.init_seeds(P);

    for (uint32_t round = 0; round < rounds; ++round) {
        for (uint32_t b = threadIdx.x; b < G.na; b += kBlockP)
            cnt[b] = 0;
        for (uint32_t i = threadIdx.x; i < kTileA; i += kBlockP)
            bkt[i] = kNoBucket;
        __syncthreads();
        if (busy) {
            for (uint32_t st = 0; st < steps; ++st) {
                bool valid = false;
                uint64_t x = 0, s = 0;
                if (walker.p < w1)
                    walker.step(valid, x, s);
                // target t of lane l goes to slot (step_base + t) * 64 + l: the
                // lanes of one LDS write hit consecutive words (no bank conflict)
                uint32_t slot = (wv * steps + st) * RE * kWave + lane;
                wave_targets<R_T, ETA_T>(P, set_ids, cache, valid, x, s, [&](uint64_t gb) {
                    const uint32_t b = (uint32_t)(gb >> shA);
                    bkt[slot] = (uint16_t)b;
                    ent[slot] = (uint32_t)(gb & maskA);
                    slot += kWave;
                    atomicAdd(&cnt[b], 1u);
                });
            }
        }
        __syncthreads();
        const uint32_t total = block_exclusive_scan(cnt, lbase, G.na, wsum);
        RunReservation res;
        res.issue(cnt, G.na, G.fillA);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kTileA; i += kBlockP) {
            const uint32_t b = bkt[i];
            if (b == kNoBucket)
                continue;
            const uint32_t pos = lbase[b] + atomicAdd(&cnt[b], 1u);
            srt[pos] = ent[i];
            sbk[pos] = (uint16_t)b;
        }
        res.finish(gbase, G.na, G.slabA, G.capA);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < total; i += kBlockP) {
            const uint32_t b = sbk[i];
            const uint32_t e = srt[i];
            const uint32_t g = gbase[b];
            if (g == kFail)
                fallback_or(P, G, ((uint64_t)b << shA) | e);
            else
                G.slabA[(uint64_t)b * G.capA + g + (i - lbase[b])] = e;
        }
        __syncthreads();
    }
}

template <int R_T, int ETA_T>
__global__ __launch_bounds__(kBlockP) void k_bin_windows(Params P, BinGeom G, const uint32_t *set_ids,
                                                         const uint64_t *offsets, uint64_t n_seqs,
                                                         const uint8_t *chars, uint64_t n_chars, uint64_t p_begin,
                                                         uint64_t p_end, uint32_t steps, uint32_t rounds)
{
    bin_generic<R_T, ETA_T, WindowWalker>(P, G, set_ids, p_begin, p_end, steps, rounds,
                                          [&](WindowWalker &w, uint64_t first, uint64_t end) {
                                              w.init(offsets, n_seqs, chars, n_chars, first, end, P.k, P.kmask);
                                          });
}

// Stage A from codes or raw keys for every shape (run-time R and eta).
__global__ __launch_bounds__(kBlockP) void k_bin_codes(Params P, BinGeom G, const uint32_t *set_ids,
                                                       const uint64_t *offsets, uint64_t n_sets,
                                                       const uint64_t *codes, uint64_t p_begin, uint64_t p_end,
                                                       uint32_t steps, uint32_t rounds)
{
    bin_generic<0, 0, CodeWalker>(P, G, set_ids, p_begin, p_end, steps, rounds,
                                  [&](CodeWalker &w, uint64_t first, uint64_t end) {
                                      w.init(offsets, n_sets, codes, first, end, P.k, P.kmask, P.raw_keys != 0,
                                             P.err);
                                  });
}

// Stage A for compile-time shapes: the targets of a round stay in registers
// instead of an unsorted LDS copy.  Each target takes its rank inside its
// bucket from the counting atomic itself, so after the scan it goes straight
// to its sorted slot: LDS holds only the sorted tile (6 bytes per target) and
// two workgroups fit a CU.
constexpr uint32_t kHoldBucketsPerThread = 4;   // the held-target kernel takes at most 2048 coarse buckets

__host__ __device__ constexpr uint32_t hold_steps(uint32_t re)
{
    return 10240u / (kBlockP * re) > 0 ? 10240u / (kBlockP * re) : 1u;
}
__host__ __device__ constexpr uint32_t hold_tile(uint32_t re) { return hold_steps(re) * kBlockP * re; }
__host__ __device__ constexpr size_t lds_bytes_stage_a_hold(uint32_t re, uint32_t na)
{
    return hold_tile(re) * 6ull + na * 12ull + 64;
}

// The body, for any walker of terms (WindowWalker over sequences,
// CodeWalker over codes or keys); init_walker(w, first, end) starts it on
// the terms [first, end).
template <int R_T, int ETA_T, class Walker, class Init>
__device__ __forceinline__ void bin_hold(const Params &P, const BinGeom &G, const uint32_t *set_ids,
                                         uint64_t p_begin, uint64_t p_end, uint32_t rounds, Init &&init_walker)
{
    constexpr uint32_t RE = R_T * ETA_T;
    constexpr uint32_t ST = hold_steps(RE);
    constexpr uint32_t TILE = hold_tile(RE);
    constexpr uint32_t NT = ST * RE;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    extern __shared__ uint32_t lds[];
    uint32_t *srt = lds;                                          // TILE: low bits of each target, sorted
    uint16_t *sbk = reinterpret_cast<uint16_t *>(srt + TILE);     // TILE: its bucket
    uint32_t *cnt = reinterpret_cast<uint32_t *>(sbk + TILE);     // na: counts (reset by the reservation)
    uint32_t *lbase = cnt + G.na;                                 // na: first sorted slot of each bucket
    uint32_t *gbase = lbase + G.na;                               // na: first slab entry of each run
    uint32_t *wsum = gbase + G.na;                                // kWavesP
    const uint32_t shA = G.rb + G.fb;
    const uint64_t maskA = (1ull << shA) - 1;
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t span = (uint64_t)rounds * ST * kWave;
    const uint64_t w0 = p_begin + ((uint64_t)blockIdx.x * kWavesP + wv) * span;
    const uint64_t w1 = min(w0 + span, p_end);
    const bool busy = w0 < p_end;
    Walker walker;
    if (busy)
        init_walker(walker, w0, w1);
    SetCache cache;
    cache.init_seeds(P);
    for (uint32_t b = threadIdx.x; b < G.na; b += kBlockP)
        cnt[b] = 0;
    __syncthreads();

    for (uint32_t round = 0; round < rounds; ++round) {
        // bucket | rank << 16 (kNone: no target) and low bits of each held target
        uint32_t hbr[NT], he[NT];
#pragma unroll
        for (uint32_t st = 0; st < ST; ++st) {
            bool valid = false;
            uint64_t x = 0, s = 0;
            if (busy && walker.p < w1)
                walker.step(valid, x, s);
            uint64_t gb[RE];
            const bool ok = window_targets<R_T, ETA_T>(P, set_ids, cache, valid, x, s, gb);
#pragma unroll
            for (uint32_t t = 0; t < RE; ++t) {
                const uint32_t b = (uint32_t)(gb[t] >> shA);
                he[st * RE + t] = (uint32_t)(gb[t] & maskA);
                hbr[st * RE + t] = ok ? (b | (atomicAdd(&cnt[b], 1u) << 16)) : kNone;
            }
        }
        __syncthreads();
        const uint32_t total = block_exclusive_scan(cnt, lbase, G.na, wsum);
        RunReservationT<kHoldBucketsPerThread> res;
        res.issue(cnt, G.na, G.fillA);
#pragma unroll
        for (uint32_t i = 0; i < NT; ++i) {
            if (hbr[i] == kNone)
                continue;
            const uint32_t b = hbr[i] & 0xFFFFu;
            const uint32_t pos = lbase[b] + (hbr[i] >> 16);
            srt[pos] = he[i];
            sbk[pos] = (uint16_t)b;
        }
        res.finish(gbase, G.na, G.slabA, G.capA);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < total; i += kBlockP) {
            const uint32_t b = sbk[i];
            const uint32_t e = srt[i];
            const uint32_t g = gbase[b];
            if (g == kFail)
                fallback_or(P, G, ((uint64_t)b << shA) | e);
            else
                G.slabA[(uint64_t)b * G.capA + g + (i - lbase[b])] = e;
        }
        // no barrier here: the next round's first barrier (after its
        // counting) is reached only when every wave has finished this loop,
        // and the counting touches only cnt, which this loop does not read
    }
}

template <int R_T, int ETA_T>
__global__ __launch_bounds__(kBlockP) __attribute__((amdgpu_waves_per_eu(4)))
void k_bin_windows_hold(Params P, BinGeom G, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_seqs,
                        const uint8_t *chars, uint64_t n_chars, uint64_t p_begin, uint64_t p_end, uint32_t rounds)
{
    bin_hold<R_T, ETA_T, WindowWalker>(P, G, set_ids, p_begin, p_end, rounds,
                                       [&](WindowWalker &w, uint64_t first, uint64_t end) {
                                           w.init(offsets, n_seqs, chars, n_chars, first, end, P.k, P.kmask);
                                       });
}

// Stage A from codes or raw keys: the terms of code q (set set_ids[s] for
// offsets[s] <= q < offsets[s+1]) instead of the windows of sequences.
template <int R_T, int ETA_T>
__global__ __launch_bounds__(kBlockP) __attribute__((amdgpu_waves_per_eu(4)))
void k_bin_codes_hold(Params P, BinGeom G, const uint32_t *set_ids, const uint64_t *offsets, uint64_t n_sets,
                      const uint64_t *codes, uint64_t p_begin, uint64_t p_end, uint32_t rounds)
{
    bin_hold<R_T, ETA_T, CodeWalker>(P, G, set_ids, p_begin, p_end, rounds,
                                     [&](CodeWalker &w, uint64_t first, uint64_t end) {
                                         w.init(offsets, n_sets, codes, first, end, P.k, P.kmask, P.raw_keys != 0,
                                                P.err);
                                     });
}

// Stage B: block = (coarse bucket, tile of TILE slots of its nwg chunks,
// which lie one after the other), BLK threads.  A slot holds an entry when
// it is below its chunk's fill count (and is not a sentinel).  The tile's
// entries stay in registers; the counting atomic gives each its rank inside
// its region, so after the scan it goes straight to its sorted LDS slot (4
// bytes of LDS per entry).  Larger tiles give longer runs per region, so
// fewer partly written memory segments.  LDS: the sorted tile, then two
// words per region (the count, which the reservation turns into the run's
// first slab entry, and the first sorted slot); the scan's wave sums use
// the tile's space before any entry is sorted into it.
template <int BLK, uint32_t TILE>
__host__ __device__ constexpr size_t lds_bytes_stage_b_t(uint32_t nf)
{
    return TILE * 4ull + nf * 8ull;
}

template <int BLK, uint32_t TILE>
__global__ __launch_bounds__(BLK) void k_bin_regions(Params P, BinGeom G, uint32_t tiles_per_bucket)
{
    extern __shared__ uint32_t lds[];
    static_assert(BLK / kWave <= TILE, "wave sums fit the tile");
    uint32_t *srt = lds;                // TILE entries sorted by region
    uint32_t *cnt = srt + TILE;         // nf counts (read and reset by the reservation) ...
    uint32_t *gbase = cnt;              // ... whose finish stores the runs' first slab entries there
    uint32_t *lbase = cnt + G.nf;       // nf first sorted slots
    uint32_t *wsum = srt;               // BLK / 64, only while the scan runs
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    // workgroup i runs on XCD i mod kXcds; the group's coarse buckets are
    // dealt to the XCDs (buckets x, x + kXcds, ... to XCD x), so every region
    // of a bucket is written through one XCD's L2, which can join the runs
    // that different tiles append next to each other
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const uint32_t cl = x + kXcds * (j / tiles_per_bucket);
    if (cl >= G.ncb)
        return;
    const uint32_t c = G.c0 + cl;
    const uint32_t tile = j % tiles_per_bucket;
    const uint64_t span = (uint64_t)G.nwg * G.capA;   // slots of bucket c
    const uint64_t t0 = (uint64_t)tile * TILE;
    if (t0 >= span)
        return;
    const uint32_t n = (uint32_t)min((uint64_t)TILE, span - t0);
    const uint32_t *cfill = G.fillA + (uint64_t)c * G.nwg;
    {
        // leave at once when no chunk holds an entry in [t0, t0 + n)
        const uint64_t g0 = t0 / G.capA, g1 = (t0 + n - 1) / G.capA;
        bool any = false;
        for (uint64_t g = g0; g <= g1 && !any; ++g)
            any = g * G.capA + min((uint64_t)cfill[g], G.capA) > t0;
        if (!any)
            return;
    }
    const uint32_t *src = G.slabA + (uint64_t)c * span + t0;   // 16-byte aligned: capA, t0 are multiples of 4
    const double inv_cap = 1.0 / (double)G.capA;
    for (uint32_t b = threadIdx.x; b < G.nf; b += BLK)
        cnt[b] = 0;
    // unconditional loads (clamped to the last vector) so none waits for
    // another; entries past n are not counted
    constexpr int kV = TILE / 4 / BLK;
    static_assert(kV * 4 * BLK == (int)TILE, "tile of whole vectors per thread");
    u32x4 v[kV];
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
    const uint32_t n4 = (n + 3) / 4;
#pragma unroll
    for (int i = 0; i < kV; ++i)
        v[i] = s4[min((uint32_t)(i * BLK) + threadIdx.x, n4 - 1)];
    // each vector's chunk (its 4 slots share one: capA is a multiple of 4)
    // and that chunk's fill, loaded for every vector before any is used so
    // that the loads are in flight together
    uint32_t gv[kV], fv[kV];
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const uint64_t p = t0 + 4ull * ((uint32_t)(i * BLK) + threadIdx.x);
        uint64_t g = 0;
        if (G.nwg > 1) {
            g = (uint64_t)((double)p * inv_cap);
            if (g * G.capA > p)
                --g;
            else if ((g + 1) * G.capA <= p)
                ++g;
        }
        gv[i] = (uint32_t)min(g, (uint64_t)G.nwg - 1);
        fv[i] = cfill[gv[i]];
    }
    // how many of each vector's slots hold entries (0..4), 4 bits per vector
    static_assert(kV <= 8, "slot counts of 4 bits fit one word");
    uint32_t nv = 0;
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const uint32_t j = (uint32_t)(i * BLK) + threadIdx.x;
        const uint64_t p = t0 + 4ull * j;
        const uint64_t end = (uint64_t)gv[i] * G.capA + min((uint64_t)fv[i], G.capA);   // past the chunk's entries
        uint32_t a = end > p ? (uint32_t)min(end - p, (uint64_t)4) : 0u;
        a = j * 4 < n ? min(a, n - j * 4) : 0u;
        nv |= a << (4 * i);
    }
    __syncthreads();
    uint32_t rk[kV * 4];
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const uint32_t e[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
        const uint32_t a = (nv >> (4 * i)) & 15u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool ok = (uint32_t)q < a && e[q] != kSentinel;
            rk[i * 4 + q] = ok ? atomicAdd(&cnt[e[q] >> G.rb], 1u) : kNone;
        }
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan<BLK>(cnt, lbase, G.nf, wsum);
    uint32_t *fill = G.fillB + (uint64_t)(c - G.c0) * G.nf;
    uint32_t *slab = G.slabB + (uint64_t)(c - G.c0) * G.nf * G.capB;
    RunReservationT<(kMaxBucketsPerThread * kBlockP + BLK - 1) / BLK, BLK> res;
    res.issue(cnt, G.nf, fill);
    // every sorted slot first (rk becomes the slot), then the LDS writes, so
    // no read waits behind a write
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const uint32_t e[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (rk[i * 4 + q] != kNone)
                rk[i * 4 + q] += lbase[e[q] >> G.rb];
    }
#pragma unroll
    for (int i = 0; i < kV; ++i) {
        const uint32_t e[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (rk[i * 4 + q] != kNone)
                srt[rk[i * 4 + q]] = e[q];
    }
    res.finish(gbase, G.nf, slab, G.capB);
    __syncthreads();
    const uint32_t maskB = (1u << G.rb) - 1;
    const uint32_t capB32 = (uint32_t)G.capB;   // below 2^31 (the scratch plan's bound)
    const uint64_t cbit = (uint64_t)c << (G.rb + G.fb);
    // kOut sorted slots per thread at a time: their LDS reads are in flight
    // together
    constexpr uint32_t kOut = 8;
    for (uint32_t i0 = threadIdx.x; i0 < total; i0 += BLK * kOut) {
        uint32_t e[kOut], g[kOut], lb[kOut];
#pragma unroll
        for (uint32_t u = 0; u < kOut; ++u) {
            const uint32_t i = i0 + u * BLK;
            e[u] = i < total ? srt[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < kOut; ++u) {
            g[u] = gbase[e[u] >> G.rb];
            lb[u] = lbase[e[u] >> G.rb];
        }
#pragma unroll
        for (uint32_t u = 0; u < kOut; ++u) {
            const uint32_t i = i0 + u * BLK;
            if (i < total) {
                if (g[u] == kFail)
                    fallback_or(P, G, cbit + e[u]);
                else
                    slab[(uint64_t)(e[u] >> G.rb) * capB32 + g[u] + (i - lb[u])] = e[u] & maskB;
            }
        }
    }
}

// Stage C: block = region of the group (global region G.c0 * nf + block).
// Regions no target reached are left untouched.  With `fresh` the index is
// known to have been all zero before this batch (nothing inserted since it
// was created or cleared): a region that no fallback atomic touched starts
// from zero in LDS instead of being read.
__global__ __launch_bounds__(kBlockC) void k_apply_regions(Params P, BinGeom G, uint32_t fresh)
{
    extern __shared__ uint32_t lds[];   // 2^rb / 32 words
    const uint64_t gl = blockIdx.x;                       // in the group's slab B
    const uint64_t g = (uint64_t)G.c0 * G.nf + gl;        // in the index
    const uint32_t rwords = 1u << (G.rb - 5);
    const uint64_t w0 = g * rwords;
    if (w0 >= G.total_words)
        return;
    const uint64_t n = min((uint64_t)G.fillB[gl], G.capB);
    if (n == 0)
        return;
    const uint32_t nw = (uint32_t)min((uint64_t)rwords, G.total_words - w0);   // a multiple of 4
    u32x4 *l4 = reinterpret_cast<u32x4 *>(lds);
    const u32x4 *g4 = reinterpret_cast<const u32x4 *>(P.index + w0);
    const uint32_t nw4 = nw / 4;
    constexpr int kRegion4PerThread = (1u << (kRegionLog2Max - 5)) / 4 / kBlockC;
    constexpr int kBatch = 8;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(G.slabB + gl * G.capB);   // capB is a multiple of 4
    const uint64_t n4 = (n + 3) / 4;
    // The region and the first batch of its targets are loaded together:
    // every load is unconditional (clamped to an in-bounds vector) so all of
    // them are in flight before the first use.
    u32x4 ev[kBatch];
    if (fresh && !G.dirty[g]) {
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            ev[i] = s4[min((uint64_t)i * kBlockC + threadIdx.x, n4 - 1)];
        const u32x4 zero = {0u, 0u, 0u, 0u};
        for (uint32_t j = threadIdx.x; j < nw4; j += kBlockC)
            l4[j] = zero;
    } else {
        u32x4 rv[kRegion4PerThread];
#pragma unroll
        for (int i = 0; i < kRegion4PerThread; ++i)
            rv[i] = g4[min((uint32_t)(i * kBlockC) + threadIdx.x, nw4 - 1)];
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            ev[i] = s4[min((uint64_t)i * kBlockC + threadIdx.x, n4 - 1)];
#pragma unroll
        for (int i = 0; i < kRegion4PerThread; ++i) {
            const uint32_t j = i * kBlockC + threadIdx.x;
            if (j < nw4)
                l4[j] = rv[i];
        }
    }
    __syncthreads();
    auto apply = [&](uint64_t j0) {
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const uint64_t j = j0 + (uint64_t)i * kBlockC + threadIdx.x;
            const uint32_t e[4] = {ev[i].x, ev[i].y, ev[i].z, ev[i].w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j * 4 + q < n && e[q] != kSentinel)
                    atomicOr(&lds[e[q] >> 5], 1u << (e[q] & 31u));
        }
    };
    apply(0);
    for (uint64_t j0 = (uint64_t)kBatch * kBlockC; j0 < n4; j0 += (uint64_t)kBatch * kBlockC) {
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            ev[i] = s4[min(j0 + (uint64_t)i * kBlockC + threadIdx.x, n4 - 1)];
        apply(j0);
    }
    __syncthreads();
    u32x4 *o4 = reinterpret_cast<u32x4 *>(P.index + w0);
    for (uint32_t i = threadIdx.x; i < nw4; i += kBlockC)
        o4[i] = l4[i];
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *p, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

// Fill n words with v: a kernel, so that a call recorded into a graph holds
// no memset node.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

}  // namespace rambo_dev
