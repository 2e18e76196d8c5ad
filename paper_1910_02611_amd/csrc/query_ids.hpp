// Answers of sequence queries as ascending set-ID lists, and per-cell fill
// counts of the index.
//
// The ID form compacts the K-bit answer of Sec. 3.2.1 (Alg. 2's A).  It
// starts from the per-read group masks that the work-queue launch leaves in
// its state (run without the mask expansion), then
//   k_ids_count : |A| per read: either the candidate members of one
//                 repetition's positive cells tested against the others, or
//                 the popcounts of the expanded K-bit words;
//   k_scan64_*  : exclusive scan of the counts into id_offsets (n+1 entries);
//   k_ids_write : the same enumeration again, writing the IDs in ascending
//                 order at their wave-prefix positions.
// Both take 64 consecutive reads per wave: the lanes check them at once and
// the wave then works through the ones with a (possibly) non-empty answer.
// A short list found by k_ids_count is kept in the read's mask words, and
// k_ids_write only copies it.
// A read whose list would end beyond the caller's capacity is not written and
// the sticky overflow bit is raised; id_offsets is always complete.
//
// k_fill_counts counts the set bits of each cell (r, b): the n_b of the
// fill 1 - (1 - 1/m)^(eta n) of Sec. 2, per BFU.
#pragma once

#include "query_queue.hpp"

namespace rambo_dev {

constexpr int kErrOverflow = 4;
constexpr uint32_t kScanTile = 1024;   // elements per block of the u64 scan (256 threads x 4)

// Whether read q's answer is known to be empty without its masks: no valid
// window, or a repetition the probing already found empty.
__device__ __forceinline__ bool read_known_empty(const ReadQueue &Q, uint64_t q)
{
    return Q.dead[q] != 0 || Q.nk[q] == 0;
}

// Loads read q's final group masks (R x SW words) into the wave's LDS G and
// tells whether some repetition has no positive cell.  The whole wave calls.
__device__ __forceinline__ bool load_read_masks(const Params &P, const ReadQueue &Q, uint64_t q, uint32_t SW,
                                                uint32_t *G, uint32_t lane)
{
    const uint32_t rsw = P.R * SW;
    for (uint32_t i = lane; i < rsw; i += kWave)
        G[i] = Q.G[q * rsw + i];
    wave_sync_lds();
    return any_rep_empty_wave(G, P.R, SW, lane);
}

// How a read's answer is enumerated.  By the partition identity, A is the
// set of members i of the positive cells of any one repetition r* with
// phi_r(i) positive in every other repetition.  When r*'s candidates times
// the other repetitions cost less than expanding all W words over every
// positive cell, the candidates are tested one by one (a few hundred for a
// large K); otherwise the K-bit words are expanded.
struct Enum {
    bool by_members;
    uint32_t rstar;      // repetition whose members are enumerated
    uint32_t cells;      // positive cells of rstar
};

// The whole wave plans in one pass over the words of every repetition: lane
// l takes words l, l + 64, ... of the R*SW.  A positive cell's candidates are
// its member count (from member_off); the counts of the first cell of four
// words per lane are loaded together before any is used, so a read whose
// words hold one positive cell each costs one round trip to memory instead
// of one per repetition.  The per-repetition sums (candidates, then positive
// cells) gather in acc, 2 R words of the wave's LDS.
__device__ __forceinline__ Enum plan_enum(const Params &P, const uint32_t *G, uint32_t SW, uint32_t lane,
                                          uint32_t *acc)
{
    const uint32_t R = P.R, rsw = R * SW;
    const uint32_t sw_log = (uint32_t)__builtin_ctz(SW);   // SW is a power of two
    for (uint32_t i = lane; i < 2 * R; i += kWave)
        acc[i] = 0;
    wave_sync_lds();
    constexpr uint32_t kU = 4;   // words per lane whose loads are in flight together
    for (uint32_t w0 = lane; w0 < rsw; w0 += kU * kWave) {
        uint32_t bits[kU], r_of[kU], lo[kU], hi[kU];
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            const uint32_t w = w0 + u * kWave;
            bits[u] = w < rsw ? G[w] : 0u;
            r_of[u] = w < rsw ? w >> sw_log : 0u;
            lo[u] = hi[u] = 0;
            if (bits[u]) {
                const uint32_t *off = P.member_off + (uint64_t)r_of[u] * (P.B + 1);
                const uint32_t b = (w - r_of[u] * SW) * 32 + (uint32_t)__builtin_ctz(bits[u]);
                lo[u] = off[b];
                hi[u] = off[b + 1];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
            if (!bits[u])
                continue;
            const uint32_t r = r_of[u];
            uint32_t cand = hi[u] - lo[u];
            // the word's further cells, one at a time
            const uint32_t *off = P.member_off + (uint64_t)r * (P.B + 1);
            const uint32_t base = (w0 + u * kWave - r * SW) * 32;
            uint32_t m = bits[u] & (bits[u] - 1);
            while (m) {
                const uint32_t b = base + (uint32_t)__builtin_ctz(m);
                m &= m - 1;
                cand += off[b + 1] - off[b];
            }
            atomicAdd(&acc[r], cand);
            atomicAdd(&acc[R + r], (uint32_t)__builtin_popcount(bits[u]));
        }
    }
    wave_sync_lds();
    Enum e{false, 0, 0};
    uint32_t best = 0xFFFFFFFFu, all_cells = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t cand = acc[r], cells = acc[R + r];
        all_cells += cells;
        if (cand < best) {
            best = cand;
            e.rstar = r;
            e.cells = cells;
        }
    }
    e.by_members = (uint64_t)best * (R - 1) <= (uint64_t)P.W * all_cells;
    return e;
}

// Whether set i is in every repetition's positive cells other than rstar.
// The first other repetition is tested alone (most candidates fail there);
// for the lanes that pass it, the cells of the remaining repetitions are
// loaded kRB at a time before any is tested, so their loads are in flight
// together.
__device__ __forceinline__ bool member_passes(const Params &P, const uint32_t *G, uint32_t SW, uint32_t rstar,
                                              uint32_t i)
{
    const uint32_t r1 = rstar == 0 ? 1u : 0u;
    if (r1 >= P.R)
        return true;
    const uint32_t b1 = P.phi[(uint64_t)r1 * P.K + i];
    if (!((G[r1 * SW + (b1 >> 5)] >> (b1 & 31)) & 1u))
        return false;
    constexpr uint32_t kRB = 4;
    bool pass = true;
    for (uint32_t r0 = r1 + 1; r0 < P.R && pass; r0 += kRB) {
        uint32_t cell[kRB];
#pragma unroll
        for (uint32_t j = 0; j < kRB; ++j) {
            const uint32_t r = r0 + j;
            cell[j] = r < P.R && r != rstar ? P.phi[(uint64_t)r * P.K + i] : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kRB; ++j) {
            const uint32_t r = r0 + j;
            if (r < P.R && r != rstar)
                pass = pass && ((G[r * SW + (cell[j] >> 5)] >> (cell[j] & 31)) & 1u);
        }
    }
    return pass;
}

// Calls f(i, pass) for the candidates of rstar, 64 at a time on the wave's
// lanes (lanes past the end get pass = false), cell by cell in ascending b.
// The words of rstar with a positive cell are found 64 at a time by a
// ballot.
template <class F>
__device__ __forceinline__ void for_candidates(const Params &P, const uint32_t *G, uint32_t SW, uint32_t rstar,
                                               uint32_t lane, F &&f)
{
    const uint32_t *off = P.member_off + (uint64_t)rstar * (P.B + 1);
    const uint32_t *mem = P.members + (uint64_t)rstar * P.K;
    for (uint32_t sw0 = 0; sw0 < SW; sw0 += kWave) {
        const uint32_t mine = sw0 + lane < SW ? G[rstar * SW + sw0 + lane] : 0u;
        uint64_t words = __ballot(mine != 0);
        while (words) {
            const uint32_t l = (uint32_t)__builtin_ctzll(words);
            words &= words - 1;
            const uint32_t sw = sw0 + l;
            uint32_t bits = G[rstar * SW + sw];
            while (bits) {
                const uint32_t b = sw * 32 + (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1;
                for (uint32_t k0 = off[b]; k0 < off[b + 1]; k0 += kWave) {
                    const uint32_t k = k0 + lane;
                    const uint32_t i = k < off[b + 1] ? mem[k] : 0u;
                    f(i, k < off[b + 1] && member_passes(P, G, SW, rstar, i));
                }
            }
        }
    }
}

// Largest list a wave sorts in LDS when the candidates come from several
// cells (their lists interleave); longer lists take the word expansion.
constexpr uint32_t kSortCap = 1024;

__device__ __forceinline__ void wave_bitonic_sort(uint32_t *a, uint32_t n_pad, uint32_t lane)
{
    for (uint32_t k = 2; k <= n_pad; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = lane; i < n_pad; i += kWave) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t x = a[i], y = a[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            wave_sync_lds();
        }
}

// A read's answer of at most min(R*SW, kSortCap) IDs is kept, ascending, in
// the read's own R*SW mask words once counted (the count kernel has the
// masks in LDS by then), so the write kernel copies it instead of
// enumerating the answer again.
__device__ __forceinline__ bool list_in_slot(uint64_t n, uint32_t rsw)
{
    return n <= rsw && n <= kSortCap;
}

// Wave per 64 consecutive reads: lane l checks read q0 + l, and only the
// reads not known to be empty are enumerated, one after the other by the
// whole wave (most reads of a batch usually are empty, and one coalesced
// check replaces a dependent load per read).  The IDs go to the wave's LDS
// buffer as they are found (sorted when they come from several cells) and,
// when the list is short enough, into the read's mask slot.
__global__ __launch_bounds__(kBlock) void k_ids_count(Params P, ReadQueue Q, uint64_t n_reads, uint32_t SW,
                                                      uint64_t *counts)
{
    extern __shared__ uint32_t lds[];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t rsw = P.R * SW;
    uint32_t *G = lds + wv * rsw;
    uint32_t *buf = lds + kWavesPerBlock * rsw + wv * kSortCap;
    const uint64_t below = (1ull << lane) - 1;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock * kWave;
    for (uint64_t q0 = ((uint64_t)blockIdx.x * kWavesPerBlock + wv) * kWave; q0 < n_reads; q0 += stride) {
        const uint64_t ql = q0 + lane;
        uint64_t todo = __ballot(ql < n_reads && !read_known_empty(Q, ql));
        uint32_t mine = 0;   // the count of read ql
        // the next read's masks are loaded while this one is enumerated
        // (reads of at most kPre * 64 mask words)
        constexpr uint32_t kPre = 3;
        const bool pre = rsw <= kPre * kWave;
        uint32_t nxt[kPre];
        auto fetch = [&](uint64_t qn) {
#pragma unroll
            for (uint32_t u = 0; u < kPre; ++u) {
                const uint32_t i = lane + u * kWave;
                nxt[u] = i < rsw ? Q.G[qn * rsw + i] : 0u;
            }
        };
        if (pre && todo)
            fetch(q0 + __builtin_ctzll(todo));
        while (todo) {
            const uint32_t l = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t q = q0 + l;
            uint32_t c = 0;
            bool empty;
            if (pre) {
#pragma unroll
                for (uint32_t u = 0; u < kPre; ++u) {
                    const uint32_t i = lane + u * kWave;
                    if (i < rsw)
                        G[i] = nxt[u];
                }
                wave_sync_lds();
                empty = any_rep_empty_wave(G, P.R, SW, lane);
                if (todo)
                    fetch(q0 + __builtin_ctzll(todo));
            } else {
                empty = load_read_masks(P, Q, q, SW, G, lane);
            }
            if (!empty) {
                const Enum e = plan_enum(P, G, SW, lane, buf);
                if (e.by_members) {
                    for_candidates(P, G, SW, e.rstar, lane, [&](uint32_t i, bool pass) {
                        const uint64_t bal = __ballot(pass);
                        const uint32_t at = c + (uint32_t)__popcll(bal & below);
                        if (pass && at < kSortCap)
                            buf[at] = i;
                        c += (uint32_t)__popcll(bal);
                    });
                    if (e.cells > 1 && list_in_slot(c, rsw)) {
                        uint32_t n_pad = 1;
                        while (n_pad < c)
                            n_pad <<= 1;
                        for (uint32_t t = c + lane; t < n_pad; t += kWave)
                            buf[t] = 0xFFFFFFFFu;
                        wave_sync_lds();
                        wave_bitonic_sort(buf, n_pad, lane);
                    }
                } else {
                    uint32_t cost;
                    const uint32_t neg = complement_reps(P, G, P.R, SW, &cost);
                    for (uint32_t w0 = 0; w0 < P.W; w0 += kWave) {
                        const uint32_t w = w0 + lane;
                        uint32_t word = w < P.W ? expand_word(P, G, SW, w, neg) : 0u;
                        const uint32_t wc = __builtin_popcount(word);
                        uint32_t at = c + wave_excl_scan_u32(wc, lane);
                        while (word) {
                            const uint32_t b = (uint32_t)__builtin_ctz(word);
                            word &= word - 1;
                            if (at < kSortCap)
                                buf[at] = w * 32 + b;
                            ++at;
                        }
                        c += wave_sum_u32(wc);
                    }
                }
                wave_sync_lds();
                if (list_in_slot(c, rsw))
                    for (uint32_t t = lane; t < c; t += kWave)
                        Q.G[q * rsw + t] = buf[t];
            }
            if (lane == l)
                mine = c;
            wave_sync_lds();
        }
        if (ql < n_reads)
            counts[ql] = mine;
    }
}

// Tile-local exclusive scan of x[0..n) into y; tile totals into part.
__global__ __launch_bounds__(256) void k_scan64_tiles(const uint64_t *x, uint64_t n, uint64_t *y, uint64_t *part)
{
    __shared__ uint64_t s[256];
    const uint32_t t = threadIdx.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * kScanTile + 4 * t;
    uint64_t v[4], sum = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = i0 + j < n ? x[i0 + j] : 0;
        sum += v[j];
    }
    s[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const uint64_t a = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint64_t run = s[t] - sum;
    for (int j = 0; j < 4; ++j) {
        if (i0 + j < n)
            y[i0 + j] = run;
        run += v[j];
    }
    if (t == 255)
        part[blockIdx.x] = s[255];
}

// One workgroup: exclusive scan of the tile totals in place; y[n] = total;
// overflow bit when the total exceeds cap.
__global__ __launch_bounds__(1024) void k_scan64_part(uint64_t *part, uint64_t nb, uint64_t *y, uint64_t n,
                                                      uint64_t cap, int *err)
{
    __shared__ uint64_t s[1024];
    const uint32_t t = threadIdx.x;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t b0 = min((uint64_t)t * per, nb), b1 = min(b0 + per, nb);
    uint64_t sum = 0;
    for (uint64_t i = b0; i < b1; ++i)
        sum += part[i];
    s[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint64_t a = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint64_t run = s[t] - sum;
    for (uint64_t i = b0; i < b1; ++i) {
        const uint64_t c = part[i];
        part[i] = run;
        run += c;
    }
    if (t == 1023) {
        y[n] = s[1023];
        if (s[1023] > cap)
            atomicOr(err, kErrOverflow);
    }
}

__global__ __launch_bounds__(256) void k_scan64_add(uint64_t *y, uint64_t n, const uint64_t *part)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        y[i] += part[i / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_ids_write(Params P, ReadQueue Q, uint64_t n_reads, uint32_t SW,
                                                      const uint64_t *id_offsets, uint32_t *ids, uint64_t cap)
{
    extern __shared__ uint32_t lds[];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    uint32_t *G = lds + wv * (P.R * SW);
    uint32_t *buf = lds + kWavesPerBlock * (P.R * SW) + wv * kSortCap;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock * kWave;
    for (uint64_t q0 = ((uint64_t)blockIdx.x * kWavesPerBlock + wv) * kWave; q0 < n_reads; q0 += stride) {
        // lane l checks read q0 + l; the reads with a list that fits are
        // written one after the other by the whole wave
        const uint64_t ql = q0 + lane;
        const uint64_t a0 = ql < n_reads ? id_offsets[ql] : 0, a1 = ql < n_reads ? id_offsets[ql + 1] : 0;
        uint64_t todo = __ballot(a1 > a0 && a1 <= cap);
        while (todo) {
            const uint32_t l = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t q = q0 + l;
            const uint64_t o0 = readlane64(a0, l), o1 = readlane64(a1, l);
            const uint32_t n = (uint32_t)(o1 - o0);
            if (list_in_slot(n, P.R * SW)) {
                // the count kernel left the list in the read's mask slot
                for (uint32_t t = lane; t < n; t += kWave)
                    ids[o0 + t] = Q.G[q * P.R * SW + t];
                continue;
            }
            load_read_masks(P, Q, q, SW, G, lane);
            const Enum e = plan_enum(P, G, SW, lane, buf);
            if (e.by_members && e.cells == 1) {
                // one member list, ascending: passing members in list order
                uint64_t base = o0;
                for_candidates(P, G, SW, e.rstar, lane, [&](uint32_t i, bool pass) {
                    const uint64_t bal = __ballot(pass);
                    if (pass)
                        ids[base + __popcll(bal & ((1ull << lane) - 1))] = i;
                    base += __popcll(bal);
                });
            } else if (e.by_members && n <= kSortCap) {
                // several lists: gather in LDS, sort, write
                uint32_t fill = 0;
                for_candidates(P, G, SW, e.rstar, lane, [&](uint32_t i, bool pass) {
                    const uint64_t bal = __ballot(pass);
                    if (pass)
                        buf[fill + __popcll(bal & ((1ull << lane) - 1))] = i;
                    fill += __popcll(bal);
                });
                uint32_t n_pad = 1;
                while (n_pad < n)
                    n_pad <<= 1;
                for (uint32_t t = n + lane; t < n_pad; t += kWave)
                    buf[t] = 0xFFFFFFFFu;
                wave_sync_lds();
                wave_bitonic_sort(buf, n_pad, lane);
                for (uint32_t t = lane; t < n; t += kWave)
                    ids[o0 + t] = buf[t];
            } else {
                uint64_t base = o0;
                uint32_t cost;
                const uint32_t neg = complement_reps(P, G, P.R, SW, &cost);
                for (uint32_t w0 = 0; w0 < P.W; w0 += kWave) {
                    const uint32_t w = w0 + lane;
                    uint32_t word = w < P.W ? expand_word(P, G, SW, w, neg) : 0u;
                    const uint32_t c = __builtin_popcount(word);
                    uint64_t pos = base + wave_excl_scan_u32(c, lane);
                    while (word) {
                        const uint32_t b = (uint32_t)__builtin_ctz(word);
                        word &= word - 1;
                        if (pos < o1)
                            ids[pos] = w * 32 + b;
                        ++pos;
                    }
                    base += wave_sum_u32(c);
                }
            }
            wave_sync_lds();
        }
    }
}

// Per-cell set-bit counts, out[r * B + b] += ones of column b in repetition
// r.  Block (x, r) takes kFillTile consecutive words of repetition r; each
// thread keeps an 8-plane vertical counter for the 32 bit positions of its
// words (all with the same position inside a row), so a word costs a few
// bitwise operations, and folds it into an LDS column histogram at the end.
constexpr uint32_t kFillWordsPerThread = 255;
constexpr uint64_t kFillTile = (uint64_t)kBlock * kFillWordsPerThread;

__global__ __launch_bounds__(kBlock) void k_fill_counts(const uint32_t *index, uint64_t words_per_rep, uint32_t S,
                                                        uint32_t B, unsigned long long *out)
{
    extern __shared__ uint32_t hist[];   // S counters
    const uint32_t r = blockIdx.y;
    const uint32_t t = threadIdx.x;
    for (uint32_t c = t; c < S; c += kBlock)
        hist[c] = 0;
    const uint32_t *rep = index + (uint64_t)r * words_per_rep;
    const uint64_t w0 = (uint64_t)blockIdx.x * kFillTile + t;
    uint32_t plane[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < kFillWordsPerThread; ++i) {
        const uint64_t w = w0 + (uint64_t)i * kBlock;
        uint32_t carry = w < words_per_rep ? rep[w] : 0u;
        for (int k = 0; k < 8; ++k) {
            const uint32_t nc = plane[k] & carry;
            plane[k] ^= carry;
            carry = nc;
        }
    }
    __syncthreads();
    // every word of this thread starts at bit (w0 * 32) mod S of its row
    const uint32_t col0 = (uint32_t)((w0 * 32) & (S - 1));
    for (uint32_t j = 0; j < 32; ++j) {
        uint32_t c = 0;
        for (int k = 0; k < 8; ++k)
            c |= ((plane[k] >> j) & 1u) << k;
        if (c)
            atomicAdd(&hist[(col0 + j) & (S - 1)], c);
    }
    __syncthreads();
    for (uint32_t c = t; c < B; c += kBlock)
        if (hist[c])
            atomicAdd(out + (uint64_t)r * B + c, (unsigned long long)hist[c]);
}

}  // namespace rambo_dev
