// Partitioned bulk insertion (Alg. 1 without global atomics).
//
// A random atomicOr per bit target is bound by the device's atomic rate, not
// by HBM bandwidth.  For bulk inserts the targets are instead partitioned by
// address, twice, and applied region by region in LDS:
//
//  A  k_bin_windows : every window's R*eta targets (global bit addresses of
//                     the bit-sliced index) are counted per coarse bucket in
//                     LDS, one run per bucket is reserved in the bucket's slab
//                     with one atomicAdd per bucket and tile, and a second
//                     pass scatters the low bits of every target into its run.
//  B  k_bin_regions : each tile of a coarse bucket's slab is split the same
//                     way into the bucket's fine buckets (index regions of
//                     2^rb bits).
//  C  k_apply_regions: one workgroup per region loads the region into LDS,
//                     ORs in its targets with LDS atomics and writes it back.
//
// OR is order-free and idempotent, so the order in which runs are filled does
// not change the index.  A run that does not fit in its slab is applied with
// global atomics instead, so every input is inserted whatever its skew.
#pragma once

#include "kernels.hpp"

namespace rambo_dev {

constexpr uint32_t kSentinel = 0xFFFFFFFFu;
constexpr uint32_t kFail = 0xFFFFFFFFu;
constexpr uint32_t kWindowsPerWaveA = 4096;     // windows per wave in stage A
constexpr uint32_t kTileB = 8192;               // slab entries per tile in stage B

struct BinGeom {
    uint32_t rb;          // log2 of the bits in one region
    uint32_t fb;          // log2 of the regions in one coarse bucket
    uint32_t na;          // coarse buckets
    uint32_t nf;          // regions per coarse bucket (1 << fb)
    uint64_t capA;        // slab entries per coarse bucket
    uint64_t capB;        // slab entries per region
    uint32_t *slabA;      // na * capA
    uint32_t *fillA;      // na
    uint32_t *slabB;      // na * nf * capB
    uint32_t *fillB;      // na * nf
    uint64_t total_words; // words of the index (all repetitions)
};

// Every target of a valid window: global bit address of (r, row, col).
template <class F>
__device__ __forceinline__ void for_each_target(const Params &P, uint64_t x, uint32_t set, F &&f)
{
    const uint64_t rep_bits = P.words_per_rep * 32;
    for (uint32_t r = 0; r < P.R; ++r) {
        const uint32_t col = P.phi[(uint64_t)r * P.K + set];
        const uint64_t base = r * rep_bits + col;
        for (uint32_t j = 0; j < P.eta; ++j)
            f(base + (bf_position(x, P.seeds[r * P.eta + j], P) << P.S_log2));
    }
}

__device__ __forceinline__ void direct_or(const Params &P, uint64_t gb)
{
    atomicOr(P.index + (gb >> 5), 1u << (gb & 31u));
}

// Reserve one run per bucket: hist[b] targets of this tile.  On success
// base[b] is the run's first slab entry and hist[b] becomes the run cursor
// (0); a run that does not fit is marked kFail and, if it starts inside the
// slab, its slab tail is filled with sentinels so readers skip it.
__device__ __forceinline__ void reserve_runs(uint32_t *hist, uint32_t *base, uint32_t nb, uint32_t *fill,
                                             uint32_t *slab, uint64_t cap)
{
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
        const uint32_t c = hist[b];
        hist[b] = 0;
        if (c == 0) {
            base[b] = kFail;
            continue;
        }
        const uint64_t pos = atomicAdd(fill + b, c);
        if (pos + c <= cap) {
            base[b] = (uint32_t)pos;
        } else {
            base[b] = kFail;
            for (uint64_t i = pos; i < cap; ++i)
                slab[(uint64_t)b * cap + i] = kSentinel;
        }
    }
}

// Stage A over the windows starting in [p_begin, p_end).
__global__ __launch_bounds__(kBlock) void k_bin_windows(Params P, BinGeom G, const uint32_t *set_ids,
                                                        const uint64_t *offsets, uint64_t n_seqs,
                                                        const uint8_t *chars, uint64_t n_chars, uint64_t p_begin,
                                                        uint64_t p_end)
{
    extern __shared__ uint32_t lds[];
    uint32_t *hist = lds;          // na counters, then run cursors
    uint32_t *base = lds + G.na;   // na run starts
    const uint32_t shA = G.rb + G.fb;
    const uint64_t maskA = (1ull << shA) - 1;
    for (uint32_t b = threadIdx.x; b < G.na; b += kBlock)
        hist[b] = 0;
    __syncthreads();

    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t w0 = p_begin + ((uint64_t)blockIdx.x * kWavesPerBlock + wv) * kWindowsPerWaveA;
    const uint64_t w1 = min(w0 + kWindowsPerWaveA, p_end);
    const bool busy = w0 < p_end;

    auto visit = [&](auto &&on_target) {
        if (!busy)
            return;
        wave_windows(offsets, n_seqs, chars, n_chars, w0, w1, P.k, P.kmask,
                     [&](uint64_t, bool valid, uint64_t x, uint64_t s) {
                         if (!valid)
                             return;
                         const uint32_t set = set_ids[s];
                         if (set >= P.K) {
                             atomicOr(P.err, kErrSetId);
                             return;
                         }
                         for_each_target(P, x, set, on_target);
                     });
    };
    // pass 1: count targets per coarse bucket
    visit([&](uint64_t gb) { atomicAdd(&hist[gb >> shA], 1u); });
    __syncthreads();
    reserve_runs(hist, base, G.na, G.fillA, G.slabA, G.capA);
    __syncthreads();
    // pass 2: the same targets again, scattered into the reserved runs
    visit([&](uint64_t gb) {
        const uint32_t b = (uint32_t)(gb >> shA);
        const uint32_t start = base[b];
        if (start == kFail) {
            direct_or(P, gb);
            return;
        }
        const uint32_t rank = atomicAdd(&hist[b], 1u);
        G.slabA[(uint64_t)b * G.capA + start + rank] = (uint32_t)(gb & maskA);
    });
}

// Stage B: block = (coarse bucket, tile of its slab).
__global__ __launch_bounds__(kBlock) void k_bin_regions(Params P, BinGeom G, uint32_t tiles_per_bucket)
{
    extern __shared__ uint32_t lds[];
    uint32_t *ent = lds;                    // kTileB entries
    uint32_t *hist = lds + kTileB;          // nf counters, then run cursors
    uint32_t *base = hist + G.nf;           // nf run starts
    const uint32_t c = blockIdx.x / tiles_per_bucket;
    const uint32_t tile = blockIdx.x % tiles_per_bucket;
    const uint64_t n_c = min((uint64_t)G.fillA[c], G.capA);
    const uint64_t t0 = (uint64_t)tile * kTileB;
    if (t0 >= n_c)
        return;
    const uint32_t n = (uint32_t)min((uint64_t)kTileB, n_c - t0);
    const uint32_t *src = G.slabA + (uint64_t)c * G.capA + t0;
    for (uint32_t b = threadIdx.x; b < G.nf; b += kBlock)
        hist[b] = 0;
    for (uint32_t i = threadIdx.x; i < n; i += kBlock)
        ent[i] = src[i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        const uint32_t e = ent[i];
        if (e != kSentinel)
            atomicAdd(&hist[e >> G.rb], 1u);
    }
    __syncthreads();
    uint32_t *fill = G.fillB + (uint64_t)c * G.nf;
    uint32_t *slab = G.slabB + (uint64_t)c * G.nf * G.capB;
    reserve_runs(hist, base, G.nf, fill, slab, G.capB);
    __syncthreads();
    const uint32_t maskB = (1u << G.rb) - 1;
    const uint64_t cbit = (uint64_t)c << (G.rb + G.fb);
    for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
        const uint32_t e = ent[i];
        if (e == kSentinel)
            continue;
        const uint32_t f = e >> G.rb;
        const uint32_t start = base[f];
        if (start == kFail) {
            direct_or(P, cbit + e);
            continue;
        }
        const uint32_t rank = atomicAdd(&hist[f], 1u);
        slab[(uint64_t)f * G.capB + start + rank] = e & maskB;
    }
}

// Stage C: block = region.  Regions no target reached are left untouched.
__global__ __launch_bounds__(kBlock) void k_apply_regions(Params P, BinGeom G)
{
    extern __shared__ uint32_t lds[];   // 2^rb / 32 words
    const uint64_t g = blockIdx.x;
    const uint64_t n = min((uint64_t)G.fillB[g], G.capB);
    if (n == 0)
        return;
    const uint32_t rwords = 1u << (G.rb - 5);
    const uint64_t w0 = g * rwords;
    if (w0 >= G.total_words)
        return;
    const uint32_t nw = (uint32_t)min((uint64_t)rwords, G.total_words - w0);   // a multiple of 4
    uint4 *l4 = reinterpret_cast<uint4 *>(lds);
    const uint4 *g4 = reinterpret_cast<const uint4 *>(P.index + w0);
    for (uint32_t i = threadIdx.x; i < nw / 4; i += kBlock)
        l4[i] = g4[i];
    __syncthreads();
    const uint32_t *src = G.slabB + g * G.capB;
    for (uint64_t i = threadIdx.x; i < n; i += kBlock) {
        const uint32_t e = src[i];
        if (e != kSentinel)
            atomicOr(&lds[e >> 5], 1u << (e & 31u));
    }
    __syncthreads();
    uint4 *o4 = reinterpret_cast<uint4 *>(P.index + w0);
    for (uint32_t i = threadIdx.x; i < nw / 4; i += kBlock)
        o4[i] = l4[i];
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t *p, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

}  // namespace rambo_dev
