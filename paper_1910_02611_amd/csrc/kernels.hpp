// RAMBO kernels for gfx950.
//
//  k_build_partition  phi_r(i) for all (r, i)                     (Alg. 1)
//  k_build_cellmask   SetIDs(M[b,r]) as K-bit masks                 (Alg. 2)
//  k_extract          canonical code of every k-window            (Sec. 3.2.1, Sec. 5.2)
//  k_insert_seqs      windows of set genomes -> atomicOr into rows (Alg. 1)
//  k_insert_kmers     k-mer codes of sets -> atomicOr into rows    (Alg. 1)
//  k_query_kmers      R*eta row gathers, AND, K-bit expansion      (Alg. 2)
//  k_query_seqs       one wave per read: AND of group masks over all windows,
//                     early exit on an empty repetition, one expansion
//                     (Sec. 3.2.1)
#pragma once

#include "device.hpp"

namespace rambo_dev {

// ---------------------------------------------------------------- set-up

struct PartitionArgs {
    uint64_t a[RAMBO_MAX_R];
    uint64_t b[RAMBO_MAX_R];
};

// (a*i + b) mod (2^61 - 1), from the 128-bit product: 2^64 = 8 (mod P) and
// 2^61 = 1 (mod P), so the high part folds in with weight 8.
__device__ __forceinline__ uint64_t affine_mod_p61(uint64_t a, uint64_t i, uint64_t b)
{
    constexpr uint64_t P = (1ull << 61) - 1;
    uint64_t lo = a * i;
    uint64_t hi = __umul64hi(a, i);
    const uint64_t lo2 = lo + b;
    hi += (lo2 < lo) ? 1u : 0u;
    lo = lo2;
    uint64_t s = (lo & P) + ((lo >> 61) | (hi << 3));
    s = (s & P) + (s >> 61);
    return s >= P ? s - P : s;
}

__global__ __launch_bounds__(kBlock) void k_build_partition(PartitionArgs A, uint32_t K, uint32_t B, uint32_t R,
                                                            uint32_t identity, uint16_t *phi)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (uint64_t)K * R)
        return;
    const uint32_t r = (uint32_t)(t / K), i = (uint32_t)(t % K);
    const uint64_t v = identity ? i : affine_mod_p61(A.a[r], i, A.b[r]);
    phi[t] = (uint16_t)(v % B);
}

// Thread (r, w) owns word w of every cell mask of repetition r.
__global__ __launch_bounds__(kBlock) void k_build_cellmask(const uint16_t *phi, uint32_t K, uint32_t B, uint32_t R,
                                                           uint32_t W, uint32_t *cellmask)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (uint64_t)R * W)
        return;
    const uint32_t r = (uint32_t)(t / W), w = (uint32_t)(t % W);
    for (uint32_t bit = 0; bit < 32; ++bit) {
        const uint32_t i = w * 32 + bit;
        if (i >= K)
            break;
        const uint32_t cell = phi[(uint64_t)r * K + i];
        cellmask[((uint64_t)r * B + cell) * W + w] |= 1u << bit;
    }
}

// ----------------------------------------------------------- folding over

// 32 bits of a repetition's bit string starting at bit `bit` (bits past the
// block read as 0).
__device__ __forceinline__ uint32_t bits32_at(const uint32_t *rep, uint64_t nwords, uint64_t bit)
{
    const uint64_t w = bit >> 5;
    const uint32_t sh = (uint32_t)(bit & 31);
    const uint32_t lo = w < nwords ? rep[w] : 0u;
    const uint32_t hi = w + 1 < nwords ? rep[w + 1] : 0u;
    return sh ? (lo >> sh) | (hi << (32 - sh)) : lo;
}

// Folding over (B -> B/2 = half): thread per word of the new index.  New
// row p, column c < half = old column c OR old column c + half of row p;
// old rows have stride S bits, new rows S2.
__global__ __launch_bounds__(kBlock) void k_fold(const uint32_t *src, uint32_t *dst, uint32_t R, uint64_t m,
                                                 uint32_t S, uint32_t S2, uint64_t wpr, uint64_t wpr2, uint32_t half)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (uint64_t)R * wpr2)
        return;
    const uint64_t r = t / wpr2, w = t % wpr2;
    const uint32_t *rep = src + r * wpr;
    uint32_t out = 0;
    if (S2 >= 32) {
        const uint64_t p = w * 32 / S2;
        const uint32_t c0 = (uint32_t)(w * 32 % S2);
        if (p < m && c0 < half) {
            uint32_t v = bits32_at(rep, wpr, p * S + c0) | bits32_at(rep, wpr, p * S + c0 + half);
            if (half - c0 < 32)
                v &= (1u << (half - c0)) - 1u;
            out = v;
        }
    } else {
        const uint32_t rpw = 32 / S2;   // rows per word; half < S2 <= 16
        for (uint32_t sl = 0; sl < rpw; ++sl) {
            const uint64_t p = w * rpw + sl;
            if (p >= m)
                break;
            const uint32_t v = (bits32_at(rep, wpr, p * S) | bits32_at(rep, wpr, p * S + half)) & ((1u << half) - 1u);
            out |= v << (sl * S2);
        }
    }
    dst[t] = out;
}

// Folding over for new rows of 32 or 64 bits (SW2 = 1 or 2 words; then
// S = 2 S2): thread per 4 words of the new index (one 16-byte store; wpr2 is
// a multiple of 4, so they share a repetition), which come from the 8 old
// words at twice their offset (two aligned 16-byte loads; a vector that
// starts past the m rows in use is not read and folds to 0).  Each old row
// as a 64- or 128-bit value V gives the new row (V | V >> half) below half.
template <int SW2>
__global__ __launch_bounds__(kBlock) void k_fold_narrow(const uint32_t *src, uint32_t *dst, uint32_t R, uint64_t m,
                                                        uint64_t wpr, uint64_t wpr2, uint32_t half)
{
    static_assert(SW2 == 1 || SW2 == 2, "narrow rows");
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t per_rep = wpr2 / 4;
    if (t >= (uint64_t)R * per_rep)
        return;
    const uint64_t r = t / per_rep, w0 = (t % per_rep) * 4;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src + r * wpr);
    const uint64_t used = 2 * m * SW2;   // old words holding rows 0 .. m-1
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const u32x4 a = 2 * w0 < used ? s4[w0 / 2] : zero;
    const u32x4 b = 2 * w0 + 4 < used ? s4[w0 / 2 + 1] : zero;
    const uint32_t o[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t v[4];
    if constexpr (SW2 == 1) {
        // S = 64, half in [17, 32]
        const uint64_t mask = (1ull << half) - 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t V = (uint64_t)o[2 * j] | ((uint64_t)o[2 * j + 1] << 32);
            v[j] = (uint32_t)((V | (V >> half)) & mask);
        }
    } else {
        // S = 128, half in [33, 64]
        const uint64_t mask = half < 64 ? (1ull << half) - 1 : ~0ull;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint64_t L = (uint64_t)o[4 * q] | ((uint64_t)o[4 * q + 1] << 32);
            const uint64_t H = (uint64_t)o[4 * q + 2] | ((uint64_t)o[4 * q + 3] << 32);
            const uint64_t hi = half < 64 ? (L >> half) | (H << (64 - half)) : H;
            const uint64_t N = (L | hi) & mask;
            v[2 * q] = (uint32_t)N;
            v[2 * q + 1] = (uint32_t)(N >> 32);
        }
    }
    reinterpret_cast<u32x4 *>(dst + r * wpr2)[w0 / 4] = u32x4{v[0], v[1], v[2], v[3]};
}

__global__ __launch_bounds__(kBlock) void k_phi_mod(uint16_t *phi, uint64_t n, uint32_t half)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < n)
        phi[t] = (uint16_t)(phi[t] % half);
}

// ------------------------------------------------------- window walking

// Cursor over the CSR of sequences: the sequence s that holds byte p.
struct SeqCursor {
    uint64_t s, beg, end;
    __device__ __forceinline__ void init(const uint64_t *offsets, uint64_t n, uint64_t p)
    {
        s = seq_of(offsets, n, p);
        beg = offsets[s];
        end = offsets[s + 1];
    }
    __device__ __forceinline__ void advance(const uint64_t *offsets, uint64_t n, uint64_t p)
    {
        while (p >= end && s + 1 < n) {
            ++s;
            beg = offsets[s];
            end = offsets[s + 1];
        }
    }
};

// Walks the windows starting at bytes [p0, p_end) of a CSR of sequences, 64
// per step: at each step lane l holds the window starting at byte p + l.
// Bytes are fetched one group (64 bytes) ahead of their use.
struct WindowWalker {
    const uint64_t *offsets;
    uint64_t n_seqs;
    const uint8_t *chars;
    uint64_t n_chars;
    uint32_t k;
    uint64_t kmask;
    uint64_t p, p_end;
    SeqCursor ca, cb;
    Group A;
    uint32_t raw_next;

    __device__ __forceinline__ uint32_t fetch(uint64_t q) const { return q < n_chars ? chars[q] : 0u; }

    __device__ __forceinline__ void classify(SeqCursor &c, uint64_t q, uint32_t raw, uint32_t &v, bool &bad,
                                             bool &st) const
    {
        c.advance(offsets, n_seqs, q);
        const bool in = q >= c.beg && q < c.end && q < n_chars;
        v = in ? base_value(raw) : 4u;
        bad = v > 3u;
        st = in && q == c.beg;
    }

    __device__ __forceinline__ void init(const uint64_t *offsets_, uint64_t n_seqs_, const uint8_t *chars_,
                                         uint64_t n_chars_, uint64_t p0, uint64_t p_end_, uint32_t k_,
                                         uint64_t kmask_)
    {
        offsets = offsets_;
        n_seqs = n_seqs_;
        chars = chars_;
        n_chars = n_chars_;
        k = k_;
        kmask = kmask_;
        p = p0;
        p_end = p_end_;
        const uint32_t lane = lane_id();
        ca.init(offsets, n_seqs, p0);
        uint32_t v;
        bool bad, st;
        classify(ca, p0 + lane, fetch(p0 + lane), v, bad, st);
        A = pack_group(v, bad, st);
        cb = ca;
        raw_next = fetch(p0 + kWave + lane);
    }

    // The next 64 windows (valid is false past p_end).  Call on every lane.
    __device__ __forceinline__ void step(bool &valid, uint64_t &canon, uint64_t &seq)
    {
        const uint32_t lane = lane_id();
        const uint32_t raw = raw_next;
        raw_next = fetch(p + 2 * kWave + lane);
        uint32_t v;
        bool bad, st;
        classify(cb, p + kWave + lane, raw, v, bad, st);
        const Group Bg = pack_group(v, bad, st);
        canon = 0;
        valid = window_code(A, Bg, lane, k, kmask, canon) && p + lane < p_end;
        seq = ca.s;
        A = Bg;
        ca = cb;
        p += kWave;
    }
};

// Walks a CSR of codes (or raw keys) [p0, p_end), 64 per step: at each step
// lane l holds the term of code p + l and the set (CSR index) it belongs to.
// Codes outside every set's range are not terms; k-mer codes >= 4^k are
// reported through err and skipped.  The same interface as WindowWalker.
struct CodeWalker {
    const uint64_t *offsets;
    uint64_t n_sets;
    const uint64_t *codes;
    uint32_t k;
    uint64_t kmask;
    bool raw;
    int *err;
    uint64_t p, p_end;
    SeqCursor c;

    __device__ __forceinline__ void init(const uint64_t *offsets_, uint64_t n_sets_, const uint64_t *codes_,
                                         uint64_t p0, uint64_t p_end_, uint32_t k_, uint64_t kmask_, bool raw_,
                                         int *err_)
    {
        offsets = offsets_;
        n_sets = n_sets_;
        codes = codes_;
        k = k_;
        kmask = kmask_;
        raw = raw_;
        err = err_;
        p = p0;
        p_end = p_end_;
        c.init(offsets, n_sets, p0);
    }

    __device__ __forceinline__ void step(bool &valid, uint64_t &x, uint64_t &seq)
    {
        const uint64_t q = p + lane_id();
        c.advance(offsets, n_sets, q);
        const bool in = q < p_end && q >= c.beg && q < c.end;
        const uint64_t code = in ? codes[q] : 0;
        const bool bad = in && !raw && code > kmask;
        if (bad)
            atomicOr(err, kErrCode);
        valid = in && !bad;
        x = raw ? code : canonical(code & kmask, k);
        seq = c.s;
        p += kWave;
    }
};

// The wave visits the windows starting at bytes [p0, p_end) and calls
// f(p, valid, canonical code, sequence) on every lane of the wave together
// (valid is false past p_end), so f may use wave-wide operations.
template <class F>
__device__ __forceinline__ void wave_windows(const uint64_t *offsets, uint64_t n_seqs, const uint8_t *chars,
                                             uint64_t n_chars, uint64_t p0, uint64_t p_end, uint32_t k,
                                             uint64_t kmask, F &&f)
{
    WindowWalker w;
    w.init(offsets, n_seqs, chars, n_chars, p0, p_end, k, kmask);
    while (w.p < p_end) {
        const uint64_t pw = w.p + lane_id();
        bool valid;
        uint64_t canon, s;
        w.step(valid, canon, s);
        f(pw, valid, canon, s);
    }
}

// One wave per chunk of `chunk` bytes (a multiple of 64).
__global__ __launch_bounds__(kBlock) void k_extract(uint32_t k, uint64_t kmask, const uint64_t *offsets,
                                                    uint64_t n_seqs, const uint8_t *chars, uint64_t n_chars,
                                                    uint64_t chunk, uint64_t *out)
{
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint64_t p0 = wave * chunk;
    if (p0 >= n_chars)
        return;
    const uint64_t pe = min(p0 + chunk, n_chars);
    wave_windows(offsets, n_seqs, chars, n_chars, p0, pe, k, kmask, [&](uint64_t p, bool valid, uint64_t canon, uint64_t) {
        if (p < pe)
            out[p] = valid ? canon : ~0ull;
    });
}

// ------------------------------------------------------------- insertion

__device__ __forceinline__ uint64_t readfirstlane64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v);
}

// The partition columns of the sequence a wave is in: lane r holds phi_r(set)
// (r < R), read back with readlane, so the hot loop issues no memory load
// for them.  Refilled only when the wave moves to another sequence.  Lane t
// also holds the position seed s_t (t = r*eta + j), filled once: reading a
// seed with readlane avoids a scalar load (and its wait, which would also
// drain pending LDS operations) per bit target.
struct SetCache {
    uint64_t s = ~0ull;
    uint32_t set = 0;
    uint32_t cols = 0;
    uint64_t seed = 0;

    __device__ __forceinline__ void init_seeds(const Params &P)
    {
        const uint32_t lane = lane_id();
#pragma unroll
        for (uint32_t t = 0; t < RAMBO_MAX_RETA; ++t)
            if (lane == t)
                seed = P.seeds[t];
    }
};

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l)
{
    return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((uint32_t)v, l);
}

// The R*eta bit targets of the window a lane holds (term x of sequence s):
// gb[t] is the global bit address in the bit-sliced index of (repetition
// t / eta, row pos_{r,j}(x), column phi_r(set)).  Returns whether this lane
// has targets (a valid window of a valid set).  When every valid lane is in
// the same sequence - the common case - the set and its columns come from the
// cache.  All R*eta hashes are independent chains (instruction-level
// parallelism for the 64-bit multiplies).  Call on every lane of the wave.
template <int R_T, int ETA_T>
__device__ __forceinline__ bool window_targets(const Params &P, const uint32_t *set_ids, SetCache &cache, bool valid,
                                               uint64_t x, uint64_t s, uint64_t (&gb)[R_T * ETA_T])
{
    const uint64_t live = __ballot(valid);
    if (!live)
        return false;
    const uint64_t rep_bits = P.words_per_rep * 32;
    const int first = __builtin_ctzll(live);
    const uint64_t s0 = readfirstlane64(__shfl(s, first, kWave));
    const bool uniform = __ballot(valid && s != s0) == 0;
    uint32_t cols[R_T];
    bool ok = valid;
    if (uniform) {
        if (s0 != cache.s) {
            cache.s = s0;
            cache.set = __builtin_amdgcn_readfirstlane(set_ids[s0]);
            const uint32_t lane = lane_id();
            cache.cols = (cache.set < P.K && lane < P.R) ? P.phi[(uint64_t)lane * P.K + cache.set] : 0u;
        }
        if (cache.set >= P.K) {
            if ((int)lane_id() == first)
                atomicOr(P.err, kErrSetId);
            return false;
        }
#pragma unroll
        for (int r = 0; r < R_T; ++r)
            cols[r] = (uint32_t)__builtin_amdgcn_readlane(cache.cols, r);
    } else {
        const uint32_t set = valid ? set_ids[s] : 0u;
        if (valid && set >= P.K)
            atomicOr(P.err, kErrSetId);
        ok = valid && set < P.K;
#pragma unroll
        for (int r = 0; r < R_T; ++r)
            cols[r] = ok ? P.phi[(uint64_t)r * P.K + set] : 0u;
    }
    const uint64_t hx = mix64(x);
#pragma unroll
    for (int t = 0; t < R_T * ETA_T; ++t)
        gb[t] = (uint64_t)(t / ETA_T) * rep_bits + cols[t / ETA_T] +
                (bf_position(hx, readlane64(cache.seed, t), P) << P.S_log2);
    return ok;
}

// Alg. 1 for the windows the wave holds: each lane with a valid window gets
// on_target(gb) for each of its R*eta bit targets (see window_targets).
// R_T == 0 is the run-time shape path.
template <int R_T, int ETA_T, class F>
__device__ __forceinline__ void wave_targets(const Params &P, const uint32_t *set_ids, SetCache &cache, bool valid,
                                             uint64_t x, uint64_t s, F &&on_target)
{
    if constexpr (R_T > 0) {
        uint64_t gb[R_T * ETA_T];
        if (window_targets<R_T, ETA_T>(P, set_ids, cache, valid, x, s, gb)) {
#pragma unroll
            for (int t = 0; t < R_T * ETA_T; ++t)
                on_target(gb[t]);
        }
        return;
    }
    const uint64_t live = __ballot(valid);
    if (!live)
        return;
    const uint64_t rep_bits = P.words_per_rep * 32;
    const uint64_t hx = mix64(x);
    const int first = __builtin_ctzll(live);
    const uint64_t s0 = readfirstlane64(__shfl(s, first, kWave));
    if (__ballot(valid && s != s0) == 0) {
        if (s0 != cache.s) {
            cache.s = s0;
            cache.set = __builtin_amdgcn_readfirstlane(set_ids[s0]);
            const uint32_t lane = lane_id();
            cache.cols = (cache.set < P.K && lane < P.R) ? P.phi[(uint64_t)lane * P.K + cache.set] : 0u;
        }
        if (cache.set >= P.K) {
            if ((int)lane_id() == first)
                atomicOr(P.err, kErrSetId);
            return;
        }
        for (uint32_t r = 0, t = 0; r < P.R; ++r) {
            const uint64_t base = r * rep_bits + (uint32_t)__builtin_amdgcn_readlane(cache.cols, r);
            for (uint32_t j = 0; j < P.eta; ++j, ++t) {
                const uint64_t seed = readlane64(cache.seed, t);
                if (valid)
                    on_target(base + (bf_position(hx, seed, P) << P.S_log2));
            }
        }
        return;
    }
    const uint32_t set = valid ? set_ids[s] : 0u;
    if (valid && set >= P.K)
        atomicOr(P.err, kErrSetId);
    const bool ok = valid && set < P.K;
    for (uint32_t r = 0, t = 0; r < P.R; ++r) {
        const uint64_t base = r * rep_bits + (ok ? P.phi[(uint64_t)r * P.K + set] : 0u);
        for (uint32_t j = 0; j < P.eta; ++j, ++t) {
            const uint64_t seed = readlane64(cache.seed, t);
            if (ok)
                on_target(base + (bf_position(hx, seed, P) << P.S_log2));
        }
    }
}

// Set one bit target with a global atomic (the result is not used, so this is
// a non-returning atomic; OR is order-free and idempotent).
__device__ __forceinline__ void direct_or(const Params &P, uint64_t gb)
{
    atomicOr(P.index + (gb >> 5), 1u << (gb & 31u));
}

// Alg. 1: every valid window of sequence s goes into the cell phi_r(set) of
// each repetition r, at its eta positions.
template <int R_T, int ETA_T>
__global__ __launch_bounds__(kBlock) void k_insert_seqs(Params P, const uint32_t *set_ids, const uint64_t *offsets,
                                                        uint64_t n_seqs, const uint8_t *chars, uint64_t n_chars,
                                                        uint64_t chunk)
{
    const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint64_t p0 = wave * chunk;
    if (p0 >= n_chars)
        return;
    const uint64_t pe = min(p0 + chunk, n_chars);
    SetCache cache;
    cache.init_seeds(P);
    wave_windows(offsets, n_seqs, chars, n_chars, p0, pe, P.k, P.kmask,
                 [&](uint64_t, bool valid, uint64_t x, uint64_t s) {
                     wave_targets<R_T, ETA_T>(P, set_ids, cache, valid, x, s,
                                              [&](uint64_t gb) { direct_or(P, gb); });
                 });
}

// Alg. 1 from codes: thread per code; the set of code c is the s with
// offsets[s] <= c < offsets[s+1].
__global__ __launch_bounds__(kBlock) void k_insert_kmers(Params P, const uint32_t *set_ids, const uint64_t *offsets,
                                                         uint64_t n_sets, const uint64_t *codes, uint64_t n_codes)
{
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t wave_first = idx - lane_id();
    if (wave_first >= n_codes)
        return;
    SeqCursor c;
    c.init(offsets, n_sets, wave_first);
    c.advance(offsets, n_sets, idx);
    if (idx >= n_codes || idx < c.beg || idx >= c.end)
        return;
    const uint32_t set = set_ids[c.s];
    const uint64_t code = codes[idx];
    if (set >= P.K) {
        atomicOr(P.err, kErrSetId);
        return;
    }
    if (code > P.kmask) {
        atomicOr(P.err, kErrCode);
        return;
    }
    const uint64_t hx = mix64(P.raw_keys ? code : canonical(code, P.k));
    for (uint32_t r = 0; r < P.R; ++r) {
        const uint32_t col = P.phi[(uint64_t)r * P.K + set];
        for (uint32_t j = 0; j < P.eta; ++j)
            set_cell_bit(P, r, bf_position(hx, P.seeds[r * P.eta + j], P), col);
    }
}

// ------------------------------------------------------------------ probe

// Group masks of the term with mix hx = mix64(x) for row words [w0, w0+L):
// g[r][.] = AND over j of row pos_{r,j}(x) of repetition r (Alg. 2, the
// filter test of every cell b of repetition r at once).  Compile-time R_T/ETA_T issue all R*eta loads
// before the first use; R_T == 0 is the run-time-sized path.
template <int SW, int L, int R_T, int ETA_T>
struct Probe {
    static constexpr int RN = R_T > 0 ? R_T : 1;
    // Fixed-size path: every load in flight at once.  Repetitions r0 ..
    // r0 + R_T - 1 go to g[0 .. R_T - 1].
    __device__ __forceinline__ static void run(const Params &P, uint64_t hx, int w0, bool ok, uint32_t (&g)[RN][L],
                                               int r0 = 0)
    {
        static_assert(R_T > 0 && ETA_T > 0, "fixed path");
        uint32_t rows[R_T * ETA_T][L];
#pragma unroll
        for (int t = 0; t < R_T * ETA_T; ++t) {
            if (ok) {
                load_row<SW, L>(P, r0 + t / ETA_T, bf_position(hx, P.seeds[r0 * ETA_T + t], P), w0, rows[t]);
            } else {
#pragma unroll
                for (int w = 0; w < L; ++w)
                    rows[t][w] = 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < R_T; ++r) {
#pragma unroll
            for (int w = 0; w < L; ++w) {
                uint32_t a = rows[r * ETA_T][w];
#pragma unroll
                for (int j = 1; j < ETA_T; ++j)
                    a &= rows[r * ETA_T + j][w];
                g[r][w] = a;
            }
        }
    }
};

// Run-time R and eta: one repetition at a time.
template <int SW, int L>
__device__ __forceinline__ void probe_rep(const Params &P, uint64_t hx, uint32_t r, int w0, bool ok, uint32_t (&acc)[L])
{
#pragma unroll
    for (int w = 0; w < L; ++w)
        acc[w] = ok ? ~0u : 0u;
    if (!ok)
        return;
    for (uint32_t j = 0; j < P.eta; ++j) {
        uint32_t row[L];
        load_row<SW, L>(P, r, bf_position(hx, P.seeds[r * P.eta + j], P), w0, row);
#pragma unroll
        for (int w = 0; w < L; ++w)
            acc[w] &= row[w];
    }
}

// K-bit answer word w from the group masks g (R x SW words, uniform across
// the lanes that share it): AND over r of the union of SetIDs(M[b,r]) over
// the cells b set in g_r (Alg. 2).
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of v over the 64 lanes (every lane gets it); call with the whole wave
// active.  The DPP pattern of wave_and: each step adds a disjoint partner
// group inside a row of 16 lanes (pairs, quads, half rows, rows), then the
// four row sums are read out.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap2, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kHalfMirror, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kMirror, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t lane)
{
    uint32_t x = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= (uint32_t)d)
            x += y;
    }
    return x - v;
}

// Bits of word x of a bit string of n bits that lie below n.
__device__ __forceinline__ uint32_t bits_below(uint32_t x, uint32_t n)
{
    const uint32_t lo = x * 32;
    return lo + 32 <= n ? ~0u : (lo >= n ? 0u : (1u << (n - lo)) - 1u);
}

// Alg. 2 takes, per repetition, the union of the sets of the positive
// cells.  The B cells of a repetition partition the K sets, so that union
// is also the complement (below K) of the union over the negative cells:
// bit r of the result says repetition r has more positive cells than
// negative ones and is built from the negative cells.  *cost: cells walked;
// *empty (when given): some repetition has no positive cell.
__device__ __forceinline__ uint32_t complement_reps(const Params &P, const uint32_t *g, uint32_t R, uint32_t SW,
                                                    uint32_t *cost, bool *empty = nullptr)
{
    uint32_t neg = 0, c = 0;
    bool none = false;
    for (uint32_t r = 0; r < R; ++r) {
        uint32_t npos = 0;
        for (uint32_t sw = 0; sw < SW; ++sw)
            npos += (uint32_t)__builtin_popcount(g[r * SW + sw]);
        none = none || npos == 0;
        if (2 * npos > P.B) {
            neg |= 1u << r;
            c += P.B - npos;
        } else {
            c += npos;
        }
    }
    *cost = c;
    if (empty)
        *empty = none;
    return neg;
}

// Expanding from the partition (K*R lookups of 2 bytes) beats walking
// `cost` cell masks of W words when cost * W exceeds K * R.
__device__ __forceinline__ bool partition_cheaper(const Params &P, uint32_t cost, uint32_t R)
{
    return (uint64_t)cost * P.W > (uint64_t)P.K * R;
}

// Word w of the answer from the group masks g (R x SW words): the AND over
// repetitions of the union of the cell masks of the positive cells, or of
// the complement of the union over the negative cells for the repetitions
// in `neg` (complement_reps).
__device__ __forceinline__ uint32_t expand_word(const Params &P, const uint32_t *g, uint32_t SW, uint32_t w,
                                                uint32_t neg)
{
    uint32_t acc = ~0u;
    for (uint32_t r = 0; r < P.R; ++r) {
        const bool c = (neg >> r) & 1u;
        uint32_t u = 0;
        for (uint32_t sw = 0; sw < SW; ++sw) {
            uint32_t bits = g[r * SW + sw];
            if (c)
                bits = ~bits & bits_below(sw, P.B);
            while (bits) {
                const uint32_t b = sw * 32 + (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1;
                u |= P.cellmask[((uint64_t)r * P.B + b) * P.W + w];
            }
        }
        acc &= c ? ~u : u;
    }
    return acc & bits_below(w, P.K);
}

__device__ __forceinline__ bool any_rep_empty(const uint32_t *g, uint32_t R, uint32_t SW)
{
    for (uint32_t r = 0; r < R; ++r) {
        uint32_t o = 0;
        for (uint32_t sw = 0; sw < SW; ++sw)
            o |= g[r * SW + sw];
        if (!o)
            return true;
    }
    return false;
}

// The same test by the whole wave (every lane gets the answer): lane l looks
// at words l, l + 64, ... (SW a power of two, R <= 16), then one wave OR.
__device__ __forceinline__ bool any_rep_empty_wave(const uint32_t *g, uint32_t R, uint32_t SW, uint32_t lane)
{
    const uint32_t sh = (uint32_t)__builtin_ctz(SW);
    uint32_t nz = 0;   // bit r: some word of repetition r is not zero
    for (uint32_t i = lane; i < R * SW; i += kWave)
        nz |= g[i] ? 1u << (i >> sh) : 0u;
    return wave_or(nz) != (1u << R) - 1u;
}

// Whether one repetition's SW words at g are all zero, by the whole wave.
__device__ __forceinline__ bool rep_empty_wave(const uint32_t *g, uint32_t SW, uint32_t lane)
{
    uint32_t o = 0;
    for (uint32_t w = lane; w < SW; w += kWave)
        o |= g[w];
    return __ballot(o != 0) == 0;
}

// Answer words from the partition instead of the cell masks: set i is in
// the answer iff its cell phi_r(i) is positive in every repetition (the
// union-then-intersection of Alg. 2, evaluated per set).  The same bits as
// the cell masks give, but the work is K*R lookups whatever the number of
// positive cells, which wins when many cells are positive and many negative
// (a term held by about half of the sets).  The whole wave takes up to NQ
// queries at once, so each phi load serves all of them: 64 sets per step, 8
// steps of loads in flight; lane l keeps word l of a 2048-set stripe of each
// query and stores it.  g[q]: query q's R x SW group-mask words, o[q] its
// answer; n <= NQ queries (wave-uniform).  R_T > 0: R fixed at compile time.
template <int R_T, int NQ>
__device__ __forceinline__ void expand_by_partition(const Params &P, const uint32_t *const (&g)[NQ], uint32_t n,
                                                    uint32_t SW, uint32_t R, uint32_t *const (&o)[NQ], uint32_t lane)
{
    constexpr int TB = 8;
    constexpr int RN = R_T > 0 ? R_T : 1;
    for (uint32_t base = 0; base < P.K; base += 64 * 32) {
        uint32_t mine[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            mine[q] = 0u;
        const uint32_t tmax = min(32u, (P.K - base + 63) / 64);
        for (uint32_t t0 = 0; t0 < tmax; t0 += TB) {
            bool valid[TB];
            uint32_t cell[TB][RN];
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                const uint32_t i = base + (t0 + u) * 64 + lane;
                valid[u] = t0 + u < tmax && i < P.K;
                if constexpr (R_T > 0) {
#pragma unroll
                    for (int r = 0; r < RN; ++r)
                        cell[u][r] = valid[u] ? P.phi[(uint64_t)r * P.K + i] : 0u;
                }
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if ((uint32_t)q >= n)
                    break;
                const uint32_t *gq = g[q];
#pragma unroll
                for (int u = 0; u < TB; ++u) {
                    bool in = valid[u];
                    if constexpr (R_T > 0) {
#pragma unroll
                        for (int r = 0; r < RN; ++r)
                            in = in && ((gq[r * SW + (cell[u][r] >> 5)] >> (cell[u][r] & 31)) & 1u);
                    } else {
                        const uint32_t i = base + (t0 + u) * 64 + lane;
                        for (uint32_t r = 0; r < R && in; ++r) {
                            const uint32_t b = P.phi[(uint64_t)r * P.K + i];
                            in = (gq[r * SW + (b >> 5)] >> (b & 31)) & 1u;
                        }
                    }
                    const uint64_t m = __ballot(in);
                    if ((lane >> 1) == t0 + u)
                        mine[q] = (lane & 1) ? (uint32_t)(m >> 32) : (uint32_t)m;
                }
            }
        }
        const uint32_t w = base / 32 + lane;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if ((uint32_t)q < n && w < P.W)
                o[q][w] = mine[q];
    }
}

template <int R_T>
__device__ __forceinline__ void expand_by_partition(const Params &P, const uint32_t *g, uint32_t SW, uint32_t R,
                                                    uint32_t *o, uint32_t lane)
{
    const uint32_t *const g1[1] = {g};
    uint32_t *const o1[1] = {o};
    expand_by_partition<R_T, 1>(P, g1, 1, SW, R, o1, lane);
}

// Cells walked per answer by expand_answer_wave (K <= 32 W, so the cell
// path is taken only with cost <= 32 R <= 512).
constexpr uint32_t kListCap = 512;
constexpr uint32_t kSegs = RAMBO_MAX_R + 1;

// One query's answer words o[0 .. W) by the whole wave from its group masks
// G (R x SW words, wave-uniform).  Zeros when empty.  Else, when the cell
// masks are less work than the partition: per repetition the shorter of its
// positive and negative cell lists goes to the wave's LDS list lst (the
// cells of repetition r at lst[seg[r] .. seg[r+1])), then every answer word
// ORs those cells' mask words (complemented for a negative list) and ANDs
// over repetitions; otherwise expand_by_partition.  lst: kListCap entries,
// seg: kSegs entries, both the wave's own.
// With defer given, a query for the partition path is not expanded here:
// *defer is set and the caller expands it (with others, sharing the loads).
template <int R_T>
__device__ __forceinline__ void expand_answer_wave(const Params &P, const uint32_t *G, uint32_t R, uint32_t SW,
                                                   bool empty, uint32_t *o, uint32_t lane, uint16_t *lst,
                                                   uint16_t *seg, bool *defer = nullptr)
{
    uint32_t cost = 0, neg = 0;
    if (!empty) {
        bool none;
        neg = complement_reps(P, G, R, SW, &cost, &none);
        empty = none;
    }
    if (empty) {
        for (uint32_t w = lane; w < P.W; w += kWave)
            o[w] = 0u;
        return;
    }
    if (cost > kListCap || partition_cheaper(P, cost, R)) {
        if (defer)
            *defer = true;
        else
            expand_by_partition<R_T>(P, G, SW, R, o, lane);
        return;
    }
    uint32_t pos = 0;
    for (uint32_t r = 0; r < R; ++r) {
        if (lane == 0)
            seg[r] = (uint16_t)pos;
        const bool c = (neg >> r) & 1u;
        for (uint32_t sw0 = 0; sw0 < SW; sw0 += kWave) {
            const uint32_t sw = sw0 + lane;
            uint32_t bits = 0;
            if (sw < SW) {
                bits = G[r * SW + sw];
                if (c)
                    bits = ~bits & bits_below(sw, P.B);
            }
            const uint32_t cnt = (uint32_t)__builtin_popcount(bits);
            uint32_t at = pos + wave_excl_scan_u32(cnt, lane);
            while (bits) {
                lst[at++] = (uint16_t)(sw * 32 + (uint32_t)__builtin_ctz(bits));
                bits &= bits - 1;
            }
            pos += wave_sum_u32(cnt);
        }
    }
    if (lane == 0)
        seg[R] = (uint16_t)pos;
    wave_sync_lds();
    if ((P.W & 3u) == 0) {
        u32x4 *o4 = reinterpret_cast<u32x4 *>(o);
        for (uint32_t w4 = lane; w4 < P.W / 4; w4 += kWave) {
            const uint32_t w = 4 * w4;
            u32x4 acc = {~0u, ~0u, ~0u, ~0u};
            for (uint32_t r = 0; r < R; ++r) {
                u32x4 u = {0u, 0u, 0u, 0u};
                const uint32_t e1 = seg[r + 1];
                for (uint32_t e = seg[r]; e < e1; ++e)
                    u |= *reinterpret_cast<const u32x4 *>(P.cellmask + ((uint64_t)r * P.B + lst[e]) * P.W + w);
                acc &= ((neg >> r) & 1u) ? ~u : u;
            }
            const u32x4 valid = {bits_below(w, P.K), bits_below(w + 1, P.K), bits_below(w + 2, P.K),
                                 bits_below(w + 3, P.K)};
            o4[w4] = acc & valid;
        }
    } else {
        for (uint32_t w = lane; w < P.W; w += kWave) {
            uint32_t acc = ~0u;
            for (uint32_t r = 0; r < R; ++r) {
                const uint32_t *m = P.cellmask + (uint64_t)r * P.B * P.W + w;
                uint32_t u = 0;
                uint32_t e = seg[r];
                const uint32_t e1 = seg[r + 1];
                // four cells at a time: their loads are in flight together
                for (; e + 4 <= e1; e += 4) {
                    const uint32_t a = m[(uint64_t)lst[e] * P.W], b = m[(uint64_t)lst[e + 1] * P.W];
                    const uint32_t c = m[(uint64_t)lst[e + 2] * P.W], d = m[(uint64_t)lst[e + 3] * P.W];
                    u |= (a | b) | (c | d);
                }
                for (; e < e1; ++e)
                    u |= m[(uint64_t)lst[e] * P.W];
                acc &= ((neg >> r) & 1u) ? ~u : u;
            }
            o[w] = acc & bits_below(w, P.K);
        }
    }
    wave_sync_lds();   // the list is the next answer's
}

// ---------------------------------------- transposed deferred answers

// A wave of k_query_kmers with rows of 8, 32 or 64 words holds QPW = 256 / SW
// terms.  Those of its terms whose answers come from the partition can be
// tested together: their group masks, transposed so that each cell of each
// repetition holds one bit per term (QPW bits: a nibble for SW = 64, a byte
// for SW = 32, a word for SW = 8), take exactly the space of the masks
// themselves, so the planes overwrite them in the wave's LDS region.  One phi
// load and R plane reads per set then serve up to eight deferred terms.

// The shapes with transposed planes: compile-time R and rows of 8, 32 or 64
// words (a word, a byte or a nibble per cell).
template <int SW, int R_T>
__host__ __device__ constexpr bool transposed_planes()
{
    return R_T > 0 && (SW == 8 || SW == 32 || SW == 64);
}

// ids[s] = the index of the s-th set bit of deferred (ascending), for the
// wave; returns the number of bits.
__device__ __forceinline__ uint32_t deferred_ids(uint64_t deferred, uint8_t *ids, uint32_t lane)
{
    if ((deferred >> lane) & 1ull)
        ids[__popcll(deferred & ((1ull << lane) - 1ull))] = (uint8_t)lane;
    wave_sync_lds();
    return (uint32_t)__popcll(deferred);
}

// Bit j of the 8-bit b to bit 4 j.
__device__ __forceinline__ uint32_t spread8_nibbles(uint32_t b)
{
    uint32_t x = b & 0xFFu;
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    return (x | (x << 3)) & 0x11111111u;
}

// Bit j of the 4-bit b to bit 8 j (the four shifted copies occupy disjoint
// bit fields, so the product has no carry).
__device__ __forceinline__ uint32_t spread4_bytes(uint32_t b) { return ((b & 0xFu) * 0x204081u) & 0x01010101u; }

// Rewrites the wave's group masks gw (term qi's R_T x SW words at
// gw + qi R_T SW) as planes: the element of cell c in repetition r (EB =
// 256 / SW bits, at element index r 32 SW + c) has bit s set iff cell c is
// positive for the s-th term of `deferred` (ascending qi).  Mask word w of
// repetition r covers cells 32 w .. 32 w + 31, whose elements fill plane
// words (r SW + w) EB .. + EB - 1.
template <int SW, int R_T>
__device__ __forceinline__ void transpose_deferred(uint32_t *gw, uint64_t deferred, uint32_t lane)
{
    constexpr uint32_t EB = 256 / SW;
    constexpr uint32_t PAIRS = R_T * SW;
    constexpr uint32_t PPL = (PAIRS + kWave - 1) / kWave;
    static_assert(EB == 4 || EB == 8 || EB == 32, "nibble, byte or word planes");
    uint32_t pl[PPL][EB];
#pragma unroll
    for (uint32_t p = 0; p < PPL; ++p) {
        const uint32_t pair = lane + p * kWave;
#pragma unroll
        for (uint32_t t = 0; t < EB; ++t)
            pl[p][t] = 0u;
        if (pair < PAIRS) {
            uint32_t s = 0;
            for (uint64_t d = deferred; d; d &= d - 1, ++s) {
                const uint32_t g = gw[(uint32_t)__builtin_ctzll(d) * PAIRS + pair];
#pragma unroll
                for (uint32_t t = 0; t < EB; ++t)
                    pl[p][t] |= (EB == 4 ? spread8_nibbles(g >> (8 * t))
                                 : EB == 8 ? spread4_bytes(g >> (4 * t))
                                           : (g >> t) & 1u)
                                << s;
            }
        }
    }
    wave_sync_lds();   // every mask is read before any plane word is written
#pragma unroll
    for (uint32_t p = 0; p < PPL; ++p) {
        const uint32_t pair = lane + p * kWave;
        if (pair < PAIRS) {
#pragma unroll
            for (uint32_t t = 0; t < EB; ++t)
                gw[pair * EB + t] = pl[p][t];
        }
    }
    wave_sync_lds();
}

// The answers of the n deferred terms from the planes (transpose_deferred):
// set i is in the answer of the s-th term iff bit s of its cell's element is
// set in every repetition (the membership test of expand_by_partition).  The
// s-th term's answer goes to out + ids[s] W.  Eight answers per pass over the
// sets; lane l keeps word l of each 2048-set stripe of each of them.
template <int SW, int R_T>
__device__ __forceinline__ void expand_planes_wave(const Params &P, const uint32_t *planes, uint32_t n, const uint8_t *ids,
                                                   uint32_t *out, uint32_t lane)
{
    constexpr uint32_t EB = 256 / SW;
    constexpr uint32_t C = 32 * SW;
    constexpr uint32_t NS = EB < 8 ? EB : 8;   // answers kept per pass
    constexpr int TB = 8;
    const uint8_t *pb = reinterpret_cast<const uint8_t *>(planes);
    for (uint32_t s0 = 0; s0 < n; s0 += NS) {
        const uint32_t ns = min(NS, n - s0);
        for (uint32_t base = 0; base < P.K; base += 64 * 32) {
            uint32_t mine[NS];
#pragma unroll
            for (uint32_t s = 0; s < NS; ++s)
                mine[s] = 0u;
            const uint32_t tmax = min(32u, (P.K - base + 63) / 64);
            for (uint32_t t0 = 0; t0 < tmax; t0 += TB) {
                bool valid[TB];
                uint32_t cell[TB][R_T];
#pragma unroll
                for (int u = 0; u < TB; ++u) {
                    const uint32_t i = base + (t0 + u) * 64 + lane;
                    valid[u] = t0 + u < tmax && i < P.K;
#pragma unroll
                    for (int r = 0; r < R_T; ++r)
                        cell[u][r] = valid[u] ? P.phi[(uint64_t)r * P.K + i] : 0u;
                }
#pragma unroll
                for (int u = 0; u < TB; ++u) {
                    if (t0 + u >= tmax)
                        break;
                    // bits above an element's own stay set: only bits s0 ..
                    // s0 + ns - 1 are tested
                    uint32_t x = valid[u] ? ~0u : 0u;
#pragma unroll
                    for (int r = 0; r < R_T; ++r) {
                        const uint32_t e = r * C + cell[u][r];
                        x &= EB == 4 ? (uint32_t)(pb[e >> 1] >> ((e & 1u) * 4u)) | 0xFFFFFFF0u
                             : EB == 8 ? (uint32_t)pb[e] | 0xFFFFFF00u
                                       : planes[e];
                    }
                    x >>= s0;
                    const bool lo = lane == 2 * (t0 + u), hi = lane == 2 * (t0 + u) + 1;
#pragma unroll
                    for (uint32_t s = 0; s < NS; ++s) {
                        if (s >= ns)
                            break;
                        const uint64_t m = __ballot((x >> s) & 1u);
                        mine[s] = lo ? (uint32_t)m : hi ? (uint32_t)(m >> 32) : mine[s];
                    }
                }
            }
            const uint32_t w = base / 32 + lane;
            if (w < P.W) {
#pragma unroll
                for (uint32_t s = 0; s < NS; ++s)
                    if (s < ns)
                        out[(uint64_t)ids[s0 + s] * P.W + w] = mine[s];
            }
        }
    }
}

// ---------------------------------------------------------- term queries

// Alg. 2 for a batch of codes.  G lanes share one query when a row is wider
// than 4 words; each lane gathers L words of each of the R*eta rows.  The
// group masks go to LDS; then sub-groups of the wave expand one query each
// into its W answer words with coalesced stores.
template <int SW, int R_T, int ETA_T>
__global__ __launch_bounds__(kBlock) void k_query_kmers(Params P, const uint64_t *codes, uint64_t n, uint32_t *out)
{
    constexpr int G = SW > 4 ? SW / 4 : 1;
    constexpr int L = SW / G;
    constexpr int QPW = kWave / G;
    constexpr int RMAX = R_T > 0 ? R_T : (int)RAMBO_MAX_R;
    __shared__ uint32_t gs[kWavesPerBlock * QPW * RMAX * SW];

    const uint32_t R = R_T > 0 ? (uint32_t)R_T : P.R;
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t ql = lane / G, part = lane % G;
    const uint64_t qbase = ((uint64_t)blockIdx.x * kWavesPerBlock + wv) * QPW;
    const uint64_t q = qbase + ql;
    uint32_t *gq = gs + (wv * QPW + ql) * RMAX * SW;

    const bool live = q < n;
    const uint64_t code = live ? codes[q] : 0;
    const bool ok = live && code <= P.kmask;
    if (live && !ok && part == 0)
        atomicOr(P.err, kErrCode);
    const uint64_t hx = mix64(P.raw_keys ? code : canonical(code & P.kmask, P.k));

    if constexpr (R_T > 0) {
        // Repetition 0 first: a term with no positive cell there has an empty
        // answer whatever the other repetitions hold (the intersection of
        // Alg. 2 is empty), so it reads no further rows.  Most absent terms
        // stop here; present terms go on with all other rows in flight.
        uint32_t g0[1][L];
        Probe<SW, L, 1, ETA_T>::run(P, hx, part * L, ok, g0);
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < L; ++w)
            any |= g0[0][w];
#pragma unroll
        for (int off = 1; off < G; off <<= 1)
            any |= __shfl_xor(any, off, kWave);
#pragma unroll
        for (int w = 0; w < L; ++w)
            gq[part * L + w] = g0[0][w];
        if constexpr (R_T > 1) {
            uint32_t g[R_T - 1][L];
            Probe<SW, L, R_T - 1, ETA_T>::run(P, hx, part * L, ok && any != 0, g, 1);
#pragma unroll
            for (int r = 1; r < R_T; ++r)
#pragma unroll
                for (int w = 0; w < L; ++w)
                    gq[r * SW + part * L + w] = g[r - 1][w];
        }
    } else {
        for (uint32_t r = 0; r < R; ++r) {
            uint32_t acc[L];
            probe_rep<SW, L>(P, hx, r, part * L, ok, acc);
#pragma unroll
            for (int w = 0; w < L; ++w)
                gq[r * SW + part * L + w] = acc[w];
        }
    }
    wave_sync_lds();

    if constexpr (SW > 4) {
        // Wide rows (few queries per wave): the whole wave expands one query
        // at a time (expand_answer_wave).
        // Answers for the partition path are deferred and then expanded
        // up to 4 at a time, sharing the phi loads.
        __shared__ uint16_t lst[kWavesPerBlock * kListCap];
        __shared__ uint16_t seg[kWavesPerBlock * kSegs];
        uint64_t deferred = 0;
        for (uint32_t qi = 0; qi < (uint32_t)QPW; ++qi) {
            const uint64_t q2 = qbase + qi;
            if (q2 >= n)
                break;
            bool d = false;
            expand_answer_wave<R_T>(P, gs + (wv * QPW + qi) * RMAX * SW, R, SW, false, out + q2 * P.W, lane,
                                    lst + wv * kListCap, seg + wv * kSegs, &d);
            if (d)
                deferred |= 1ull << qi;
        }
        if constexpr (transposed_planes<SW, R_T>()) {
            // all the wave's deferred terms together, from transposed planes
            if (deferred) {
                __shared__ uint8_t dids[kWavesPerBlock][QPW];
                const uint32_t nd = deferred_ids(deferred, dids[wv], lane);
                uint32_t *gw = gs + wv * QPW * RMAX * SW;
                transpose_deferred<SW, R_T>(gw, deferred, lane);
                expand_planes_wave<SW, R_T>(P, gw, nd, dids[wv], out + qbase * P.W, lane);
            }
            return;
        }
        constexpr int NQ = 4;
        while (deferred) {
            const uint32_t *gq[NQ];
            uint32_t *oq[NQ];
            uint32_t k = 0;
            for (; k < (uint32_t)NQ && deferred; ++k) {
                const uint32_t qi = (uint32_t)__builtin_ctzll(deferred);
                deferred &= deferred - 1;
                gq[k] = gs + (wv * QPW + qi) * RMAX * SW;
                oq[k] = out + (qbase + qi) * P.W;
            }
            for (uint32_t j = k; j < (uint32_t)NQ; ++j) {
                gq[j] = gq[0];
                oq[j] = oq[0];
            }
            const uint32_t *const (&gc)[NQ] = gq;
            uint32_t *const (&oc)[NQ] = oq;
            expand_by_partition<R_T, NQ>(P, gc, k, SW, R, oc, lane);
        }
        return;
    }

    // Narrow rows: per query, empty (some repetition has no positive cell),
    // or expanded from the cell masks (positive cells, or the complement of
    // the negative ones per repetition: nm), or from the partition when that
    // is less work (expand_by_partition).  Bit qi of ne / by_part.
    __shared__ uint32_t nm[kWavesPerBlock * QPW];
    uint32_t neg = 0, cost = 0;
    for (uint32_t r = 0; r < R; ++r) {
        uint32_t npos = 0;
#pragma unroll
        for (int w = 0; w < L; ++w)
            npos += (uint32_t)__builtin_popcount(gq[r * SW + part * L + w]);
#pragma unroll
        for (int off = 1; off < G; off <<= 1)
            npos += (uint32_t)__shfl_xor((int)npos, off, kWave);
        if (2 * npos > P.B) {
            neg |= 1u << r;
            cost += P.B - npos;
        } else {
            cost += npos;
        }
    }
    if (part == 0)
        nm[wv * QPW + ql] = neg;
    const uint64_t heavy_g = __ballot(live && part == 0 && partition_cheaper(P, cost, R));
    wave_sync_lds();
    const uint32_t ql2 = lane < (uint32_t)QPW ? lane : 0u;
    const bool nonempty = lane < (uint32_t)QPW && qbase + lane < n &&
                          !any_rep_empty(gs + (wv * QPW + ql2) * RMAX * SW, R, SW);
    const uint64_t ne = __ballot(nonempty);
    const uint64_t by_part = ne & __ballot(lane < (uint32_t)QPW && ((heavy_g >> (lane * G)) & 1));

    if ((P.W & 3u) == 0) {
        // The wave's answers are QPW * W consecutive words: each lane takes 4
        // of them (one 16-byte store) per step.  Empty answers are zeros;
        // the others OR 16-byte slices of the cell masks.
        const uint32_t W4 = P.W / 4;
        const uint64_t n_here = min((uint64_t)QPW, n - qbase);
        const uint32_t total4 = (uint32_t)n_here * W4;
        u32x4 *o4 = reinterpret_cast<u32x4 *>(out + qbase * P.W);
        for (uint32_t i = lane; i < total4; i += kWave) {
            const uint32_t qi = i / W4, w = (i - qi * W4) * 4;
            if ((by_part >> qi) & 1)
                continue;
            u32x4 acc = {0u, 0u, 0u, 0u};
            if ((ne >> qi) & 1) {
                const uint32_t *g2 = gs + (wv * QPW + qi) * RMAX * SW;
                const uint32_t negq = nm[wv * QPW + qi];
                acc = ~acc;
                for (uint32_t r = 0; r < R; ++r) {
                    const bool c = (negq >> r) & 1u;
                    u32x4 u = {0u, 0u, 0u, 0u};
                    for (uint32_t sw = 0; sw < (uint32_t)SW; ++sw) {
                        uint32_t bits = g2[r * SW + sw];
                        if (c)
                            bits = ~bits & bits_below(sw, P.B);
                        while (bits) {
                            const uint32_t b = sw * 32 + (uint32_t)__builtin_ctz(bits);
                            bits &= bits - 1;
                            u |= *reinterpret_cast<const u32x4 *>(P.cellmask + ((uint64_t)r * P.B + b) * P.W + w);
                        }
                    }
                    acc &= c ? ~u : u;
                }
                const u32x4 valid = {bits_below(w, P.K), bits_below(w + 1, P.K), bits_below(w + 2, P.K),
                                     bits_below(w + 3, P.K)};
                acc &= valid;
            }
            o4[i] = acc;
        }
        for (uint64_t bp = by_part; bp; bp &= bp - 1) {
            const uint32_t qi = (uint32_t)__builtin_ctzll(bp);
            expand_by_partition<R_T>(P, gs + (wv * QPW + qi) * RMAX * SW, SW, R, out + (qbase + qi) * P.W, lane);
        }
        return;
    }
    // Expansion: sub-groups of WG lanes, one query per sub-group at a time.
    uint32_t WG = 1;
    while (WG < P.W && WG < (uint32_t)kWave)
        WG <<= 1;
    const uint32_t nsg = kWave / WG, sg = lane / WG, wl = lane % WG;
    for (uint32_t qi = sg; qi < (uint32_t)QPW; qi += nsg) {
        const uint64_t q2 = qbase + qi;
        if (q2 >= n)
            break;
        if ((by_part >> qi) & 1)
            continue;
        const uint32_t *g2 = gs + (wv * QPW + qi) * RMAX * SW;
        const bool empty = !((ne >> qi) & 1);
        const uint32_t negq = nm[wv * QPW + qi];
        uint32_t *o = out + q2 * P.W;
        for (uint32_t w = wl; w < P.W; w += WG)
            o[w] = empty ? 0u : expand_word(P, g2, SW, w, negq);
    }
    for (uint64_t bp = by_part; bp; bp &= bp - 1) {
        const uint32_t qi = (uint32_t)__builtin_ctzll(bp);
        expand_by_partition<R_T>(P, gs + (wv * QPW + qi) * RMAX * SW, SW, R, out + (qbase + qi) * P.W, lane);
    }
}

// ------------------------------------------------------ sequence queries

// One 64-window step of a read over rows wider than 4 words (compile-time R
// and eta).  GL = SW/4 lanes share a window, each loading one 16-byte slice
// of every row, so a load instruction reads whole rows of 64/GL windows and
// each row's bytes are used at once; GL such rounds cover the step's
// windows.  The windows' mixes and validity move to the sharing lanes by
// shuffles.  Repetition 0 goes first (a read with no cell left there is
// finished); then the other repetitions, all rows of a round in flight.
// The per-slice ANDs are reduced over the lanes of the same slice and
// folded into G (R x SW words of LDS); dead is set when some repetition is
// empty.  Only the first n_it rounds run: a caller whose valid lanes are
// the first WPI n_it ones (a short term set) skips the empty rounds.  PH
// restricts the step to repetition 0 (kStepFirst) or to the others
// (kStepRest).
constexpr int kStepAll = 0, kStepFirst = 1, kStepRest = 2;

template <int SW, int R_T, int ETA_T, int PH = kStepAll>
__device__ __forceinline__ void probe_step_wide(const Params &P, uint64_t hx, bool valid, uint32_t *G, bool &dead,
                                                uint32_t lane, int n_it = SW / 4)
{
    constexpr int GL = SW / 4, WPI = kWave / GL;
    static_assert(GL >= 2 && GL * 4 == SW, "wide rows");
    const uint32_t part = lane % GL, sub = lane / GL;
    const uint32_t hx_lo = (uint32_t)hx, hx_hi = (uint32_t)(hx >> 32), ok_in = valid ? 1u : 0u;
    auto window = [&](int it, uint64_t &h, bool &ok) {
        const int src = it * WPI + (int)sub;
        h = ((uint64_t)(uint32_t)__shfl((int)hx_hi, src, kWave) << 32) | (uint32_t)__shfl((int)hx_lo, src, kWave);
        ok = __shfl((int)ok_in, src, kWave) != 0;
    };
    auto slice = [&](uint32_t r, uint64_t h, int j) {
        const uint64_t row = bf_position(h, P.seeds[r * ETA_T + j], P);
        return *reinterpret_cast<const u32x4 *>(P.index + (uint64_t)r * P.words_per_rep + row * SW + part * 4);
    };
    auto reduce = [&](u32x4 v) {
        for (int off = GL; off < kWave; off <<= 1) {
            v.x &= (uint32_t)__shfl_xor((int)v.x, off, kWave);
            v.y &= (uint32_t)__shfl_xor((int)v.y, off, kWave);
            v.z &= (uint32_t)__shfl_xor((int)v.z, off, kWave);
            v.w &= (uint32_t)__shfl_xor((int)v.w, off, kWave);
        }
        return v;
    };
    const u32x4 ones = {~0u, ~0u, ~0u, ~0u};
    if constexpr (PH != kStepRest) {
        u32x4 acc0 = ones;
#pragma unroll 4
        for (int it = 0; it < n_it; ++it) {
            uint64_t h;
            bool ok;
            window(it, h, ok);
            u32x4 a = ones;
            if (ok) {
#pragma unroll
                for (int j = 0; j < ETA_T; ++j)
                    a &= slice(0, h, j);
            }
            acc0 &= a;
        }
        acc0 = reduce(acc0);
        if (sub == 0) {
            G[part * 4 + 0] &= acc0.x;
            G[part * 4 + 1] &= acc0.y;
            G[part * 4 + 2] &= acc0.z;
            G[part * 4 + 3] &= acc0.w;
        }
        wave_sync_lds();
        if (rep_empty_wave(G, SW, lane)) {
            dead = true;
            return;
        }
        if constexpr (PH == kStepFirst)
            return;
    }
    if constexpr (R_T > 1) {
        u32x4 acc[R_T - 1];
#pragma unroll
        for (int r = 0; r < R_T - 1; ++r)
            acc[r] = ones;
#pragma unroll 2
        for (int it = 0; it < n_it; ++it) {
            uint64_t h;
            bool ok;
            window(it, h, ok);
            if (ok) {
                u32x4 rows[R_T - 1][ETA_T];
#pragma unroll
                for (int r = 1; r < R_T; ++r)
#pragma unroll
                    for (int j = 0; j < ETA_T; ++j)
                        rows[r - 1][j] = slice(r, h, j);
#pragma unroll
                for (int r = 1; r < R_T; ++r)
#pragma unroll
                    for (int j = 0; j < ETA_T; ++j)
                        acc[r - 1] &= rows[r - 1][j];
            }
        }
#pragma unroll
        for (int r = 1; r < R_T; ++r) {
            const u32x4 v = reduce(acc[r - 1]);
            if (sub == 0) {
                uint32_t *g = G + r * SW + part * 4;
                g[0] &= v.x;
                g[1] &= v.y;
                g[2] &= v.z;
                g[3] &= v.w;
            }
        }
    }
    wave_sync_lds();
    dead = any_rep_empty_wave(G, R_T, SW, lane);
}

// One step of Sec. 3.2.1: the group masks of the wave's terms (one per lane,
// mixed: hx; valid where the lane holds a term) ANDed over the lanes and into
// the running masks G (R x SW words of LDS, wave-private); dead once some
// repetition is empty (the first conclusive FALSE).  Repetition 0 first:
// once its running AND has no cell left the answer is empty (the
// intersection of Alg. 2), so the rows of the other repetitions are read
// only while it has one.  PH = kStepFirst reads repetition 0 only (dead when
// it is empty), kStepRest the others only.
template <int SW, int R_T, int ETA_T, int PH = kStepAll>
__device__ __forceinline__ void and_terms_step(const Params &P, uint64_t hx, bool valid, uint32_t *G, bool &dead,
                                               uint32_t lane, uint32_t n_valid = kWave)
{
    constexpr int L = SW < 4 ? SW : 4;
    constexpr int NSL = SW / L;
    if constexpr (R_T > 0 && SW >= 8) {
        // n_valid: the valid lanes are among the first n_valid
        constexpr uint32_t WPI = kWave / (SW / 4);
        probe_step_wide<SW, R_T, ETA_T, PH>(P, hx, valid, G, dead, lane, (int)((n_valid + WPI - 1) / WPI));
    } else if constexpr (R_T > 0) {
        if constexpr (PH != kStepRest) {
#pragma unroll 1
            for (int sl = 0; sl < NSL; ++sl) {
                uint32_t g0[1][L];
                Probe<SW, L, 1, ETA_T>::run(P, hx, sl * L, valid, g0);
#pragma unroll
                for (int w = 0; w < L; ++w) {
                    const uint32_t a = wave_and(valid ? g0[0][w] : ~0u);
                    if (lane == 0)
                        G[sl * L + w] &= a;
                }
            }
            wave_sync_lds();
            if (rep_empty_wave(G, SW, lane)) {
                dead = true;
                return;
            }
            if constexpr (PH == kStepFirst)
                return;
        }
        if constexpr (R_T > 1) {
#pragma unroll 1
            for (int sl = 0; sl < NSL; ++sl) {
                uint32_t g[R_T - 1][L];
                Probe<SW, L, R_T - 1, ETA_T>::run(P, hx, sl * L, valid, g, 1);
#pragma unroll
                for (int r = 1; r < R_T; ++r)
#pragma unroll
                    for (int w = 0; w < L; ++w) {
                        const uint32_t a = wave_and(valid ? g[r - 1][w] : ~0u);
                        if (lane == 0)
                            G[r * SW + sl * L + w] &= a;
                    }
            }
        }
        wave_sync_lds();
        dead = any_rep_empty_wave(G, R_T, SW, lane);
    } else {
        const uint32_t r0 = PH == kStepRest ? 1u : 0u, r1 = PH == kStepFirst ? 1u : P.R;
#pragma unroll 1
        for (int sl = 0; sl < NSL; ++sl) {
            for (uint32_t r = r0; r < r1; ++r) {
                uint32_t acc[L];
                probe_rep<SW, L>(P, hx, r, sl * L, valid, acc);
#pragma unroll
                for (int w = 0; w < L; ++w) {
                    const uint32_t a = wave_and(valid ? acc[w] : ~0u);
                    if (lane == 0)
                        G[r * SW + sl * L + w] &= a;
                }
            }
        }
        wave_sync_lds();
        dead = PH == kStepFirst ? rep_empty_wave(G, SW, lane) : any_rep_empty_wave(G, P.R, SW, lane);
    }
}

// Sec. 3.2.1 for the windows of one read (bytes end at pe) that start in
// [p_start, p_stop): each step takes 64 windows (one per lane), gathers their
// rows, ANDs the group masks over the lanes and into the running masks G
// (R x SW words of LDS, wave-private), and stops probing once some repetition
// is empty (the first conclusive FALSE).  Valid windows are still counted, in
// nk, to the end of the range.
//
// The windows go in blocks of kHashSteps steps.  The block's window mixes
// are computed first and kept in LDS (hc: kHashSteps x 64 mixes, vc:
// kHashSteps validity ballots, both wave-private); then repetition 0 is
// probed over the whole block, and the other repetitions after it.  Over
// rows of 8 words or more, a first look at repetition 0 over the windows of
// one probing round (kWave / (SW / 4) of them) spread evenly over the block
// comes before: a substitution or an absent k-mer rules out the up to k
// windows that cover it, so with spacing below k such a read usually ends
// there.  The AND does not depend on the order (a row read twice changes
// nothing), so only the rows read differ.
constexpr uint32_t kHashSteps = 4;

template <int SW, int R_T, int ETA_T>
__device__ __forceinline__ void read_windows_and(const Params &P, const uint8_t *chars, uint64_t pe,
                                                 uint64_t p_start, uint64_t p_stop, uint32_t *G, uint32_t &nk,
                                                 bool &dead, uint64_t *hc, uint64_t *vc)
{
    const uint32_t lane = lane_id();
    const uint64_t kmask = P.kmask;
    const uint32_t R = R_T > 0 ? (uint32_t)R_T : P.R;
    auto read_byte = [&](uint64_t p, uint32_t &v, bool &bad) {
        v = p < pe ? base_value(chars[p]) : 4u;
        bad = v > 3u;
    };
    uint32_t v;
    bool bad;
    read_byte(p_start + lane, v, bad);
    Group A = pack_group(v, bad, false);
    for (uint64_t pb = p_start; pb < p_stop; pb += (uint64_t)kHashSteps * kWave) {
        uint32_t n_st = 0;
        for (uint64_t p = pb; p < p_stop && n_st < kHashSteps; p += kWave, ++n_st) {
            read_byte(p + kWave + lane, v, bad);
            const Group Bg = pack_group(v, bad, false);
            uint64_t x = 0;
            const bool valid = (p + lane < p_stop) && window_code(A, Bg, lane, P.k, kmask, x);
            const uint64_t bal = __ballot(valid);
            nk += (uint32_t)__popcll(bal);
            A = Bg;
            if (!dead) {
                hc[n_st * kWave + lane] = mix64(x);
                if (lane == 0)
                    vc[n_st] = bal;
            }
        }
        if (dead)
            continue;
        wave_sync_lds();
        if constexpr (R_T > 0 && SW >= 8) {
            constexpr uint32_t WPI = kWave / (SW / 4);
            const uint32_t nw = (uint32_t)min<uint64_t>((uint64_t)n_st * kWave, p_stop - pb);
            const uint32_t j = lane < WPI && WPI > 1 ? lane * (nw - 1) / (WPI - 1) : 0u;
            const bool ok = lane < WPI && ((vc[j / kWave] >> (j % kWave)) & 1u) != 0;
            and_terms_step<SW, R_T, ETA_T, kStepFirst>(P, hc[j], ok, G, dead, lane, WPI);
        }
        for (uint32_t st = 0; st < n_st && !dead; ++st)
            and_terms_step<SW, R_T, ETA_T, kStepFirst>(P, hc[st * kWave + lane], ((vc[st] >> lane) & 1u) != 0, G,
                                                       dead, lane);
        if (R > 1)
            for (uint32_t st = 0; st < n_st && !dead; ++st)
                and_terms_step<SW, R_T, ETA_T, kStepRest>(P, hc[st * kWave + lane], ((vc[st] >> lane) & 1u) != 0,
                                                          G, dead, lane);
        // the next block rewrites hc and vc only after every lane has read
        // them here
        wave_sync_lds();
    }
}

// Sec. 3.2.1: one wave per read.  The read is expanded once: by the partition
// identity, AND over k-mers of the expanded answers equals the expansion of
// the AND of the group masks.  Without a mask output the window count, an
// empty flag and the group masks of a read not known to be empty are stored
// in the per-read state instead (ID-list form).
template <int SW, int R_T, int ETA_T>
__global__ __launch_bounds__(kBlock) void k_query_seqs(Params P, const uint64_t *offsets, uint64_t n_reads,
                                                       const uint8_t *chars, uint64_t n_chars, uint32_t *out,
                                                       uint32_t *out_nk, uint32_t *state_G, uint32_t *state_nk,
                                                       uint32_t *state_dead)
{
    constexpr int RMAX = R_T > 0 ? R_T : (int)RAMBO_MAX_R;
    __shared__ uint32_t Gs[kWavesPerBlock][RMAX * SW];
    __shared__ uint64_t hcs[kWavesPerBlock][kHashSteps * kWave];
    __shared__ uint64_t vcs[kWavesPerBlock][kHashSteps];

    const uint32_t R = R_T > 0 ? (uint32_t)R_T : P.R;
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t q = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    if (q >= n_reads)
        return;
    uint32_t *G = Gs[wv];
    for (uint32_t i = lane; i < R * SW; i += kWave)
        G[i] = ~0u;
    wave_sync_lds();

    uint64_t p0 = offsets[q];
    const uint64_t pe = min(offsets[q + 1], n_chars);
    if (p0 > pe)
        p0 = pe;
    uint32_t nk = 0;
    bool dead = false;
    read_windows_and<SW, R_T, ETA_T>(P, chars, pe, p0, pe, G, nk, dead, hcs[wv], vcs[wv]);
    if (out_nk && lane == 0)
        out_nk[q] = nk;
    if (!out) {
        // ID-list form: the count, whether the answer is known to be empty,
        // and (only when it is not) the final group masks go to the per-read
        // state that the ID kernels read
        const bool empty = dead || nk == 0;
        if (!empty)
            for (uint32_t i = lane; i < R * SW; i += kWave)
                state_G[q * R * SW + i] = G[i];
        if (lane == 0) {
            state_nk[q] = nk;
            state_dead[q] = empty ? 1u : 0u;
        }
        return;
    }
    __shared__ uint16_t lst[kWavesPerBlock * kListCap];
    __shared__ uint16_t seg[kWavesPerBlock * kSegs];
    expand_answer_wave<R_T>(P, G, R, SW, dead || nk == 0, out + q * P.W, lane, lst + wv * kListCap,
                            seg + wv * kSegs);
}

// Term sets per wave of k_query_termsets: one, or for rows of 32 and 64
// words with compile-time R as many as a wave of k_query_kmers holds, so that
// the sets whose answers come from the partition are tested together
// (transpose_deferred, expand_planes_wave).
template <int SW, int R_T>
__host__ __device__ constexpr uint32_t termsets_per_wave()
{
    return transposed_planes<SW, R_T>() ? 256u / SW : 1u;
}

// Sec. 3.2.1 for sets of terms given as codes (or raw keys): the answer of
// term set q, the codes codes[offsets[q] .. offsets[q+1]), holds the sets
// that hold every one of its terms.  A wave takes termsets_per_wave sets one
// after the other, 64 terms per step: the group masks are ANDed over the
// terms (stopping at the first empty repetition), then each set is expanded
// once.  An empty term set gets an empty answer; a k-mer code >= 4^k raises
// kErrCode and empties its set's answer (its own answer is empty).
template <int SW, int R_T, int ETA_T>
__global__ __launch_bounds__(kBlock) void k_query_termsets(Params P, const uint64_t *offsets, uint64_t n_sets,
                                                           const uint64_t *codes, uint64_t n_codes, uint32_t *out)
{
    constexpr int RMAX = R_T > 0 ? R_T : (int)RAMBO_MAX_R;
    constexpr uint32_t SPW = termsets_per_wave<SW, R_T>();
    __shared__ uint32_t Gs[kWavesPerBlock * SPW * RMAX * SW];
    __shared__ uint16_t lst[kWavesPerBlock * kListCap];
    __shared__ uint16_t seg[kWavesPerBlock * kSegs];

    const uint32_t R = R_T > 0 ? (uint32_t)R_T : P.R;
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t qbase = ((uint64_t)blockIdx.x * kWavesPerBlock + wv) * SPW;
    if (qbase >= n_sets)
        return;
    uint32_t *gw = Gs + wv * SPW * RMAX * SW;
    uint32_t empty = 0;   // bit qi: set qbase + qi answers the empty set
    for (uint32_t qi = 0; qi < SPW; ++qi) {
        const uint64_t q = qbase + qi;
        if (q >= n_sets)
            break;
        uint32_t *G = gw + qi * RMAX * SW;
        for (uint32_t i = lane; i < R * SW; i += kWave)
            G[i] = ~0u;
        wave_sync_lds();
        uint64_t p0 = offsets[q];
        const uint64_t pe = min(offsets[q + 1], n_codes);
        if (p0 > pe)
            p0 = pe;
        bool dead = false;
        for (uint64_t p = p0; p < pe; p += kWave) {
            const bool live = p + lane < pe;
            const uint64_t code = live ? codes[p + lane] : 0;
            const bool bad = live && code > P.kmask;
            if (bad)
                atomicOr(P.err, kErrCode);
            dead = dead || __ballot(bad) != 0;
            if (!dead)
                and_terms_step<SW, R_T, ETA_T>(P, mix64(P.raw_keys ? code : canonical(code & P.kmask, P.k)), live,
                                               G, dead, lane, (uint32_t)min(pe - p, (uint64_t)kWave));
        }
        if (dead || pe == p0)
            empty |= 1u << qi;
    }
    uint64_t deferred = 0;
    for (uint32_t qi = 0; qi < SPW; ++qi) {
        const uint64_t q = qbase + qi;
        if (q >= n_sets)
            break;
        bool d = false;
        expand_answer_wave<R_T>(P, gw + qi * RMAX * SW, R, SW, (empty >> qi) & 1u, out + q * P.W, lane,
                                lst + wv * kListCap, seg + wv * kSegs, SPW > 1 ? &d : nullptr);
        if (d)
            deferred |= 1ull << qi;
    }
    if constexpr (SPW > 1) {
        if (deferred) {
            __shared__ uint8_t dids[kWavesPerBlock][SPW];
            const uint32_t nd = deferred_ids(deferred, dids[wv], lane);
            transpose_deferred<SW, R_T>(gw, deferred, lane);
            expand_planes_wave<SW, R_T>(P, gw, nd, dids[wv], out + qbase * P.W, lane);
        }
    }
}

}  // namespace rambo_dev
