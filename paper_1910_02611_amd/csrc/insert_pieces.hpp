// Stage A of the partitioned insert over sequence pieces (compile-time R and
// eta): the binning kernel for sequence input.
//
// Work unit: a piece = up to kPieceWindows consecutive windows of ONE
// sequence, so a wave's set and partition columns are the same for all of
// its lanes.  Lane l of the wave holding a piece takes the piece's windows
// l*L .. l*L + L - 1 (L = kPieceLaneWindows) and walks them with a rolling
// 2-bit code: each byte shifts into the forward code and the reverse
// complement, a run counter of valid bases tells when a full window ends
// (any byte other than ACGTacgt resets it).  Bytes come from dword-aligned
// 32-byte blocks, one block ahead of their use.
//
// Binning: the workgroup is persistent over a contiguous range of the
// batch's pieces and owns a private chunk of every coarse bucket's slab
// (chunk (b, g) of ccap entries for workgroup g).  Each round the waves
// count their targets per bucket in LDS (the counting atomic returns each
// target's rank), one scan gives the tile's sorted layout, every target
// goes straight to its sorted LDS slot, and the sorted tile is written out
// run by run, each run appended at the workgroup's cursor in the bucket's
// chunk; no global atomic reserves anything.  At exit each workgroup stores
// how many entries each of its chunks holds.  A run that no
// longer fits its chunk is applied with global atomics (the region marked so
// that stage C reads it back), as in the other stage-A kernels.
#pragma once

#include "insert_part.hpp"

namespace rambo_dev {

constexpr uint32_t kPieceLaneWindows = 128;                     // L
constexpr uint32_t kPieceWindows = kWave * kPieceLaneWindows;   // windows per piece
constexpr uint32_t kPieceDummy = 64;   // per-lane counters that sort the lanes' invalid targets past the valid ones
constexpr int kBlockPc = 1024;          // workgroup of the piece kernel (one per CU: 4 waves per SIMD)
constexpr int kWavesPc = kBlockPc / kWave;

struct PieceArgs {
    const uint32_t *set_ids;
    const uint64_t *offsets;       // n_seqs + 1 byte offsets of the sequences (from the caller's chars)
    uint64_t n_seqs;
    const uint8_t *chars;          // the caller's bytes, moved down to a 4-byte boundary
    uint64_t n_bytes;              // readable bytes from `chars` (the caller's n_chars + mis)
    uint32_t mis;                  // the caller's chars start `mis` bytes after `chars`
    const uint32_t *piece_first;   // n_seqs + 1: first piece of each sequence, [n_seqs] = all pieces
    uint64_t q_begin, q_end;       // the batch's pieces
};

// Pieces of each sequence: ceil(windows / kPieceWindows); thread per sequence.
__global__ __launch_bounds__(kBlock) void k_piece_counts(const uint64_t *offsets, uint64_t n_seqs, uint64_t n_chars,
                                                         uint32_t k, uint32_t *piece_first)
{
    const uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n_seqs)
        return;
    const uint64_t b = min(offsets[s], n_chars), e = min(offsets[s + 1], n_chars);
    const uint64_t len = e > b ? e - b : 0;
    const uint64_t nw = len >= k ? len - k + 1 : 0;
    piece_first[s] = (uint32_t)((nw + kPieceWindows - 1) / kPieceWindows);
}

// 16 bytes at byte offset a of the readable range.  Past its end only whole
// dwords that hold a readable byte are loaded (the 4-byte word that holds
// the last byte lies in the same page as that byte); the rest reads as 0.
__device__ __forceinline__ u32x4 load_block(const uint8_t *base, uint64_t n_bytes, uint64_t a)
{
    if (a + 16 <= n_bytes)
        return *reinterpret_cast<const u32x4 *>(base + a);
    const uint32_t *w = reinterpret_cast<const uint32_t *>(base + a);
    return u32x4{a < n_bytes ? w[0] : 0u, a + 4 < n_bytes ? w[1] : 0u, a + 8 < n_bytes ? w[2] : 0u,
                 a + 12 < n_bytes ? w[3] : 0u};
}

// A lane's bytes in order, from 32-byte blocks loaded one block ahead of
// their use.  (Reading a loaded register waits for every older memory
// operation of the wave, the stores of the binning included, so blocks are
// large: one such wait per 32 bytes.)  The buffer state (counts, dword
// index) is the same on every lane - all lanes take a byte at once and start
// at the same offset within a dword - so refills are uniform branches.
struct ByteFeed {
    u32x4 c0, c1, n0, n1;   // current block, next block
    uint64_t buf;           // bytes not yet taken, lowest first
    uint32_t nb;            // bytes in buf (uniform)
    uint32_t di;            // next dword pair of the current block: 0..3 (uniform)
    uint64_t next_a;        // byte offset of the block after the next one

    __device__ __forceinline__ void start(const uint8_t *base, uint64_t n_bytes, uint64_t first, uint32_t skip)
    {
        // first is 4-byte aligned; skip (< 4, uniform) leading bytes are dropped
        c0 = load_block(base, n_bytes, first);
        c1 = load_block(base, n_bytes, first + 16);
        n0 = load_block(base, n_bytes, first + 32);
        n1 = load_block(base, n_bytes, first + 48);
        next_a = first + 64;
        di = 0;
        refill(base, n_bytes);
        buf >>= 8 * skip;
        nb = 8 - skip;
    }
    __device__ __forceinline__ void refill(const uint8_t *base, uint64_t n_bytes)
    {
        // selects, not a switch: every case is one dword pair of the block
        const uint32_t d = __builtin_amdgcn_readfirstlane(di);
        const bool upper = (d & 2u) != 0, odd = (d & 1u) != 0;
        const uint32_t lo0 = odd ? c0.z : c0.x, hi0 = odd ? c0.w : c0.y;
        const uint32_t lo1 = odd ? c1.z : c1.x, hi1 = odd ? c1.w : c1.y;
        const uint32_t lo = upper ? lo1 : lo0, hi = upper ? hi1 : hi0;
        buf = (uint64_t)lo | ((uint64_t)hi << 32);
        nb = 8;
        di = (__builtin_amdgcn_readfirstlane(di) + 1) & 3u;
        if (di == 0) {
            c0 = n0;
            c1 = n1;
            n0 = load_block(base, n_bytes, next_a);
            n1 = load_block(base, n_bytes, next_a + 16);
            next_a += 32;
        }
    }
    __device__ __forceinline__ uint32_t take(const uint8_t *base, uint64_t n_bytes)
    {
        if (__builtin_amdgcn_readfirstlane(nb) == 0)
            refill(base, n_bytes);
        const uint32_t c = (uint32_t)buf & 0xFFu;
        buf >>= 8;
        nb = __builtin_amdgcn_readfirstlane(nb) - 1;
        return c;
    }
};

// Rolling k-mer state of one lane: forward code, reverse-complement code and
// the number of valid bases in a row.
struct Rolling {
    uint64_t fwd, rc;
    uint32_t run;

    // One more byte: A/a 0, C/c 1, G/g 2, T/t 3 shift in; any other byte
    // resets the run.  (For the four letters, bits 1-2 of the byte XOR-ed
    // give the base value: A 0x41 -> 0, C 0x43 -> 1, G 0x47 -> 2, T 0x54 -> 3,
    // and the same for lower case.)
    __device__ __forceinline__ void push(uint32_t c, uint64_t kmask, uint32_t rc_shift)
    {
        const uint32_t d = (c | 0x20u) - 0x61u;   // 'a' -> 0, 'c' -> 2, 'g' -> 6, 't' -> 19
        const bool ok = d < 20u && ((0x80045u >> d) & 1u);
        const uint32_t v = ((c >> 1) ^ (c >> 2)) & 3u;
        run = ok ? run + 1 : 0u;
        fwd = ((fwd << 2) | v) & kmask;
        rc = (rc >> 2) | ((uint64_t)(v ^ 3u) << rc_shift);
    }
    __device__ __forceinline__ uint64_t canon() const { return fwd < rc ? fwd : rc; }
};

// Exclusive scan of cnt[0..nb) into lbase[0..nb) by the workgroup, then, for
// the real buckets b < na, the destination of this round's run of b in the
// workgroup's chunk (dst[b] = chunk slot of sorted position 0, so sorted
// position i goes to dst[b] + i; kFail64 when the run no longer fits) and the
// chunk cursor.  Resets cnt.  Returns the number of valid targets (the
// sorted positions below lbase[na]).  Ends with a barrier.
constexpr uint64_t kFail64 = ~0ull;

__device__ __forceinline__ uint32_t piece_round_scan(uint32_t *cnt, uint32_t *lbase, uint32_t *cur, uint64_t *dst,
                                                     uint32_t *wsum, uint32_t na, uint64_t chunk0, uint64_t bstride,
                                                     uint64_t ccap)
{
    const uint32_t nb = na + kPieceDummy;
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t per = (nb + kBlockPc - 1) / kBlockPc;
    const uint32_t b0 = min(threadIdx.x * per, nb), b1 = min(b0 + per, nb);
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
    uint32_t wbase = 0;
#pragma unroll
    for (int w = 0; w < kWavesPc; ++w)
        wbase += (uint32_t)w < wv ? wsum[w] : 0u;
    uint32_t run = wbase + incl - s;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t c = cnt[b];
        lbase[b] = run;
        if (b < na) {
            const uint32_t st = cur[b];
            if ((uint64_t)st + c <= ccap) {
                dst[b] = chunk0 + (uint64_t)b * bstride + st - run;
                cur[b] = st + c;
            } else {
                dst[b] = kFail64;
            }
        }
        cnt[b] = 0;
        run += c;
    }
    __syncthreads();
    return lbase[na];
}

template <int R_T, int ETA_T, int ST>
__host__ __device__ constexpr uint32_t piece_tile()
{
    return (uint32_t)ST * kBlockPc * R_T * ETA_T;
}

template <int R_T, int ETA_T, int ST>
__host__ __device__ constexpr size_t lds_bytes_pieces(uint32_t na)
{
    // sorted tile (u32 entry + u16 bucket), counters and sorted bases of the
    // na + kPieceDummy buckets, cursors and 64-bit run destinations of the
    // na real ones, wave sums
    return (size_t)piece_tile<R_T, ETA_T, ST>() * 6 + (size_t)(na + kPieceDummy) * 8 + (size_t)na * 12 + 64;
}

// FAST: m is a power of two of at most 2^32 and every repetition is a whole
// number of coarse buckets (shA <= 31), so a target's bucket and entry come
// from 32-bit arithmetic on its position; otherwise the general 64-bit form.
template <int R_T, int ETA_T, int ST, bool FAST>
__global__ __launch_bounds__(kBlockPc) __attribute__((amdgpu_waves_per_eu(4)))
void k_bin_pieces(Params P, BinGeom G, PieceArgs A)
{
    constexpr uint32_t RE = R_T * ETA_T;
    constexpr uint32_t NT = ST * RE;
    constexpr uint32_t TILE = piece_tile<R_T, ETA_T, ST>();
    constexpr uint32_t ROUNDS = kPieceLaneWindows / ST;
    static_assert(kPieceLaneWindows % ST == 0, "rounds per piece");
    static_assert(TILE <= 65536, "ranks are 16-bit");
    extern __shared__ uint32_t lds[];
    const uint32_t na = G.na;
    uint32_t *srt = lds;                                                 // TILE
    uint16_t *sbk = reinterpret_cast<uint16_t *>(srt + TILE);            // TILE
    uint64_t *dst = reinterpret_cast<uint64_t *>(sbk + TILE);            // na (8-byte aligned: TILE is even)
    uint32_t *cnt = reinterpret_cast<uint32_t *>(dst + na);              // na + dummy
    uint32_t *lbase = cnt + na + kPieceDummy;                            // na + dummy
    uint32_t *cur = lbase + na + kPieceDummy;                            // na
    uint32_t *wsum = cur + na;                                           // kWavesPc

    const uint32_t wg = blockIdx.x, nwg = gridDim.x;
    const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
    const uint32_t shA = G.rb + G.fb;
    const uint64_t rep_bits = P.words_per_rep * 32;
    const uint32_t k = P.k;
    // this workgroup's pieces
    const uint64_t total = A.piece_first[A.n_seqs];
    const uint64_t qe = min(A.q_end, total);
    const uint64_t nq = qe > A.q_begin ? qe - A.q_begin : 0;
    const uint64_t qa = A.q_begin + nq * wg / nwg, qz = A.q_begin + nq * (wg + 1) / nwg;

    for (uint32_t b = threadIdx.x; b < na + kPieceDummy; b += kBlockPc)
        cnt[b] = 0;
    for (uint32_t b = threadIdx.x; b < na; b += kBlockPc)
        cur[b] = 0;
    __syncthreads();

    for (uint64_t q0 = qa; q0 < qz; q0 += kWavesPc) {
        // the wave's piece: sequence s (the last one whose first piece is <= q)
        const uint64_t q = q0 + wv;
        bool live = q < qz;
        uint64_t s = 0;
        if (live) {
            uint64_t lo = 0, hi = A.n_seqs;   // piece_first[lo] <= q < piece_first[hi]
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) >> 1;
                if (A.piece_first[mid] <= q)
                    lo = mid;
                else
                    hi = mid;
            }
            s = lo;
        }
        s = readfirstlane64(s);
        uint64_t seq_beg = 0, nw = 0, j = 0;
        uint32_t set = 0;
        if (live) {
            seq_beg = min(A.offsets[s], A.n_bytes - A.mis);
            const uint64_t e = min(A.offsets[s + 1], A.n_bytes - A.mis);
            const uint64_t len = e > seq_beg ? e - seq_beg : 0;
            nw = len >= k ? len - k + 1 : 0;
            j = q - A.piece_first[s];
            set = A.set_ids[s];
            if (set >= P.K) {
                if (lane == 0)
                    atomicOr(P.err, kErrSetId);
                live = false;
            }
        }
        // the set's column in each repetition
        uint32_t col[R_T];
#pragma unroll
        for (uint32_t r = 0; r < R_T; ++r)
            col[r] = live ? P.phi[(uint64_t)r * P.K + set] : 0u;
        // the lane's windows: first window wl of the sequence, nl of them
        const uint64_t wl = j * kPieceWindows + (uint64_t)lane * kPieceLaneWindows;
        const uint32_t nl = live && wl < nw ? (uint32_t)min<uint64_t>(nw - wl, kPieceLaneWindows) : 0u;
        const uint64_t first = nl ? seq_beg + A.mis + wl : 0;   // the lane's first byte in A.chars
        ByteFeed feed;
        feed.start(A.chars, A.n_bytes, first & ~3ull, (uint32_t)((seq_beg + A.mis) & 3u));
        Rolling roll{0, 0, 0};
        const uint64_t kmask = P.kmask;
        const uint32_t rc_shift = 2 * k - 2;
        for (uint32_t i = 0; i + 1 < k; ++i)
            roll.push(feed.take(A.chars, A.n_bytes), kmask, rc_shift);

        for (uint32_t round = 0; round < ROUNDS; ++round) {
            uint32_t hbr[NT], he[NT];
#pragma unroll
            for (uint32_t st = 0; st < ST; ++st) {
                roll.push(feed.take(A.chars, A.n_bytes), kmask, rc_shift);
                const bool valid = roll.run >= k && round * ST + st < nl;
                const uint64_t hx = mix64(roll.canon());
#pragma unroll
                for (uint32_t t = 0; t < RE; ++t) {
                    const uint32_t r = t / ETA_T;
                    uint32_t b, e;
                    if constexpr (FAST) {
                        // position: the top m_log2 bits of (mult * hx) mod 2^64,
                        // i.e. of its high word; bucket and entry of bit
                        // pos * S + col of repetition r
                        const uint32_t mlo = (uint32_t)P.seeds[t], mhi = (uint32_t)(P.seeds[t] >> 32);
                        const uint32_t hlo = (uint32_t)hx, hhi = (uint32_t)(hx >> 32);
                        const uint32_t h32 = __umulhi(mlo, hlo) + mlo * hhi + mhi * hlo;
                        const uint32_t pos = h32 >> (32u - P.m_log2);
                        const uint32_t sh1 = shA - P.S_log2;
                        b = (uint32_t)((uint64_t)r * rep_bits >> shA) + (pos >> sh1);
                        e = ((pos & ((1u << sh1) - 1u)) << P.S_log2) | col[r];
                    } else {
                        const uint64_t gb =
                            (uint64_t)r * rep_bits + col[r] + (bf_position(hx, P.seeds[t], P) << P.S_log2);
                        b = (uint32_t)(gb >> shA);
                        e = (uint32_t)gb & (uint32_t)((1ull << shA) - 1);
                    }
                    b = valid ? b : na + lane;
                    he[st * RE + t] = e;
                    hbr[st * RE + t] = b | (atomicAdd(&cnt[b], 1u) << 16);
                }
            }
            __syncthreads();
            const uint32_t total_valid = piece_round_scan(cnt, lbase, cur, dst, wsum, na, (uint64_t)wg * G.capA,
                                                          (uint64_t)nwg * G.capA, G.capA);
            // every sorted slot first (hbr becomes slot | bucket << 16), then
            // the LDS writes, so no read waits behind a write
#pragma unroll
            for (uint32_t i = 0; i < NT; ++i) {
                const uint32_t b = hbr[i] & 0xFFFFu;
                hbr[i] = (lbase[b] + (hbr[i] >> 16)) | (b << 16);
            }
#pragma unroll
            for (uint32_t i = 0; i < NT; ++i) {
                srt[hbr[i] & 0xFFFFu] = he[i];
                sbk[hbr[i] & 0xFFFFu] = (uint16_t)(hbr[i] >> 16);
            }
            __syncthreads();
            // kOut sorted slots per thread at a time: their LDS reads are in
            // flight together
            constexpr uint32_t kOut = 4;
            for (uint32_t i0 = threadIdx.x; i0 < total_valid; i0 += kBlockPc * kOut) {
                uint32_t b[kOut], e[kOut];
                uint64_t d[kOut];
#pragma unroll
                for (uint32_t u = 0; u < kOut; ++u) {
                    const uint32_t i = i0 + u * kBlockPc;
                    b[u] = i < total_valid ? sbk[i] : 0u;
                    e[u] = i < total_valid ? srt[i] : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < kOut; ++u)
                    d[u] = dst[b[u]];
#pragma unroll
                for (uint32_t u = 0; u < kOut; ++u) {
                    const uint32_t i = i0 + u * kBlockPc;
                    if (i < total_valid) {
                        if (d[u] != kFail64)
                            G.slabA[d[u] + i] = e[u];
                        else
                            fallback_or(P, G, ((uint64_t)b[u] << shA) | e[u]);
                    }
                }
            }
            // no barrier here: the next round's counting touches only cnt
            // (reset by the scan), and its scan, which rewrites lbase and
            // dst, comes after a barrier every wave reaches only once it has
            // left this loop
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < na; b += kBlockPc)
        G.fillA[(uint64_t)b * nwg + wg] = cur[b];
}

}  // namespace rambo_dev
