// Batched sequence queries with a work queue (Sec. 3.2.1 over a batch of
// reads of uneven length in one persistent launch).
//
//  k_rq_setup   : thread per read: its number of chunks (of `chunk` bytes),
//                 per-read state (running group masks = all ones, window
//                 count, early-exit flag, chunks left), work counter = 0.
//  k_rq_scan    : one workgroup: exclusive scan of the chunk counts, so that
//                 work item i is chunk i - items[q] of the read q with
//                 items[q] <= i < items[q+1].
//  k_rq_persist : a fixed grid of waves pops items from the counter; each
//                 runs its chunk's windows (probe, AND, early exit), ANDs the
//                 result into the read's state with atomics and raises the
//                 read's flag when some repetition is empty in the chunk, so
//                 later chunks of that read only count windows.  The wave that finishes a
//                 read's last chunk expands it and writes the answer (unless
//                 no mask output is given: then the final group masks stay in
//                 the state for the ID-list kernels).
#pragma once

#include "kernels.hpp"

namespace rambo_dev {

struct ReadQueue {
    uint32_t *G;           // n_reads x (R*SW): running group masks
    uint32_t *nk;          // n_reads: valid windows
    uint32_t *dead;        // n_reads: some repetition is empty
    uint32_t *remaining;   // n_reads: chunks not yet finished
    uint32_t *items;       // n_reads + 1: first work item of each read, then the total
    uint32_t *counter;     // next work item
};

__device__ __forceinline__ void read_span(const uint64_t *offsets, uint64_t q, uint64_t n_chars, uint64_t &p0,
                                          uint64_t &pe)
{
    p0 = offsets[q];
    pe = min(offsets[q + 1], n_chars);
    if (p0 > pe)
        p0 = pe;
}

// The number of reads of a batch: n_host, or *n_dev when given (a captured
// graph replays the same launches for batches of any size up to its grid).
__device__ __forceinline__ uint64_t batch_reads(uint64_t n_host, const uint64_t *n_dev)
{
    return n_dev ? *n_dev : n_host;
}

__global__ __launch_bounds__(kBlock) void k_rq_setup(ReadQueue Q, const uint64_t *offsets, uint64_t n_host,
                                                     const uint64_t *n_dev, uint64_t n_chars, uint32_t chunk,
                                                     uint32_t rsw)
{
    const uint64_t n_reads = batch_reads(n_host, n_dev);
    const uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q == 0)
        *Q.counter = 0;
    if (q >= n_reads)
        return;
    uint64_t p0, pe;
    read_span(offsets, q, n_chars, p0, pe);
    const uint64_t len = pe - p0;
    const uint32_t chunks = len == 0 ? 1u : (uint32_t)((len + chunk - 1) / chunk);
    Q.items[q] = chunks;
    Q.remaining[q] = chunks;
    Q.nk[q] = 0;
    Q.dead[q] = 0;
    for (uint32_t i = 0; i < rsw; ++i)
        Q.G[q * rsw + i] = ~0u;
}

// Exclusive scan of items[0..n) in place, items[n] = total; one workgroup.
__global__ __launch_bounds__(1024) void k_rq_scan(uint32_t *items, uint64_t n_host, const uint64_t *n_dev)
{
    __shared__ uint32_t part[1024];
    const uint64_t n = batch_reads(n_host, n_dev);
    const uint32_t t = threadIdx.x;
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t b0 = min((uint64_t)t * per, n), b1 = min(b0 + per, n);
    uint32_t s = 0;
    for (uint64_t i = b0; i < b1; ++i)
        s += items[i];
    part[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (uint64_t i = b0; i < b1; ++i) {
        const uint32_t c = items[i];
        items[i] = run;
        run += c;
    }
    if (t == 1023)
        items[n] = part[1023];
}

// Last q with items[q] <= item (items strictly increasing: every read has a chunk).
__device__ __forceinline__ uint64_t read_of_item(const uint32_t *items, uint64_t n_reads, uint32_t item)
{
    uint64_t lo = 0, hi = n_reads;
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (items[mid] <= item)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <int SW, int R_T, int ETA_T>
__global__ __launch_bounds__(kBlock) void k_rq_persist(Params P, ReadQueue Q, const uint64_t *offsets,
                                                       uint64_t n_host, const uint64_t *n_dev, const uint8_t *chars,
                                                       uint64_t n_chars, uint32_t chunk, uint32_t *out,
                                                       uint32_t *out_nk)
{
    const uint64_t n_reads = batch_reads(n_host, n_dev);
    constexpr int RMAX = R_T > 0 ? R_T : (int)RAMBO_MAX_R;
    __shared__ uint32_t Gs[kWavesPerBlock][RMAX * SW];
    __shared__ uint64_t hcs[kWavesPerBlock][kHashSteps * kWave];
    __shared__ uint64_t vcs[kWavesPerBlock][kHashSteps];
    const uint32_t R = R_T > 0 ? (uint32_t)R_T : P.R;
    const uint32_t rsw = R * SW;
    const uint32_t lane = lane_id();
    uint32_t *G = Gs[threadIdx.x / kWave];
    __shared__ uint16_t lst[kWavesPerBlock * kListCap];
    __shared__ uint16_t seg[kWavesPerBlock * kSegs];
    uint16_t *my_lst = lst + (threadIdx.x / kWave) * kListCap, *my_seg = seg + (threadIdx.x / kWave) * kSegs;
    const uint32_t total = Q.items[n_reads];

    for (;;) {
        // the pop is made by the wave's first active lane and broadcast from
        // it, so every lane of the wave sees the same item even if control
        // flow ever reached this point with some lanes off: a pop by a fixed
        // lane that is off would leave the others on a stale item, never
        // reaching the exit test below
        const bool leader = lane == (uint32_t)__builtin_ctzll(__ballot(1));
        uint32_t item = 0;
        if (leader)
            item = atomicAdd(Q.counter, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total)
            break;
        const uint64_t q = read_of_item(Q.items, n_reads, item);
        const uint32_t c = item - Q.items[q];
        uint64_t p0, pe;
        read_span(offsets, q, n_chars, p0, pe);
        const uint64_t ps = min(p0 + (uint64_t)c * chunk, pe), pstop = min(ps + chunk, pe);

        for (uint32_t i = lane; i < rsw; i += kWave)
            G[i] = ~0u;
        wave_sync_lds();
        const bool was_dead = __hip_atomic_load(Q.dead + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        bool dead = was_dead;
        uint32_t nk = 0;
        read_windows_and<SW, R_T, ETA_T>(P, chars, pe, ps, pstop, G, nk, dead, hcs[threadIdx.x / kWave],
                                         vcs[threadIdx.x / kWave]);

        if (lane == 0 && nk)
            atomicAdd(Q.nk + q, nk);
        if (!was_dead) {
            // AND this chunk's masks into the read's (a word of all ones
            // changes nothing); a repetition empty in the chunk empties the
            // read
            for (uint32_t i = lane; i < rsw; i += kWave) {
                const uint32_t mine = G[i];
                if (mine != ~0u)
                    atomicAnd(Q.G + q * rsw + i, mine);
            }
            if (dead && lane == 0)
                atomicOr(Q.dead + q, 1u);
        }
        uint32_t left = 0;
        if (lane == (uint32_t)__builtin_ctzll(__ballot(1)))
            left = __hip_atomic_fetch_sub(Q.remaining + q, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        left = __builtin_amdgcn_readfirstlane(left);
        if (left != 1)
            continue;
        // last chunk of read q: every other chunk's AND happened before its
        // release-decrement, which our acquire-decrement follows
        const uint32_t nk_all = __hip_atomic_load(Q.nk + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (out_nk && lane == 0)
            out_nk[q] = nk_all;
        if (!out)
            continue;   // the answer stays in the state (ID-list form)
        for (uint32_t i = lane; i < rsw; i += kWave)
            G[i] = __hip_atomic_load(Q.G + q * rsw + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wave_sync_lds();
        expand_answer_wave<R_T>(P, G, R, SW, nk_all == 0, out + q * P.W, lane, my_lst, my_seg);
        wave_sync_lds();
    }
}

}  // namespace rambo_dev
