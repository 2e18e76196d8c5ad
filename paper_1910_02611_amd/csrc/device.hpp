// Device-side building blocks of the RAMBO kernels (gfx950, wave64).
//
// Hashing and encoding follow the conventions stated in include/rambo.h.
// This file is the GPU library's own implementation of them; nothing here
// is shared with any other implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rambo.h"

namespace rambo_dev {

// Four packed 32-bit words: one 16-byte vector load or store.  (A native
// vector type keeps register arrays of them in registers.)
using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // four waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// Device error bits (sticky flag of the handle).
constexpr int kErrSetId = 1;
constexpr int kErrCode = 2;

// Everything a kernel needs to address the index; passed by value.
struct Params {
    uint32_t *index;            // R blocks of words_per_rep words
    const uint16_t *phi;        // phi_r(i) at [r*K + i]
    const uint32_t *cellmask;   // SetIDs(M[b,r]) as K-bit masks at [(r*B + b)*W + w]
    const uint32_t *member_off; // SetIDs(M[b,r]) as ascending lists: members[member_off[r*(B+1) + b] ..
    const uint32_t *members;    //   member_off[r*(B+1) + b + 1]) of repetition r's block (K entries)
    int *err;                   // sticky error bits
    uint64_t m;                 // Bloom-filter positions per repetition
    uint64_t words_per_rep;
    uint64_t kmask;             // 4^k - 1
    uint32_t K, B, R, eta, k, W;
    uint32_t S_log2;            // log2 of the row stride in bits
    uint32_t m_log2;            // log2(m) when m is a power of two, else 0
    uint32_t raw_keys;          // 1: terms are 64-bit keys taken as they are (no canonical k-mer form)
    uint32_t rep_first;         // bit t: probe t is the first of its repetition
    uint32_t rep_last;          // bit t: probe t is the last of its repetition
    uint8_t rep_of[RAMBO_MAX_RETA];    // repetition of probe t = r*eta + j
    uint64_t seeds[RAMBO_MAX_RETA];    // odd multipliers s_{r,j} | 1 at t = r*eta + j
};

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// splitmix64's output function (Steele, Lea, Flood 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Bloom-filter position (Sec. 2, eta universal hashes per filter): the
// multiply-shift family over hx = mix64(x), the term's bijective mix computed
// once per term.  mult is the odd multiplier of (repetition, hash):
// floor(((mult * hx) mod 2^64) * m / 2^64), the top log2(m) bits of the
// product when m is a power of two.
__device__ __forceinline__ uint64_t bf_position(uint64_t hx, uint64_t mult, const Params &P)
{
    const uint64_t v = mult * hx;
    return P.m_log2 ? (v >> (64u - P.m_log2)) : __umul64hi(v, P.m);
}

// Base value of one byte: A/a 0, C/c 1, G/g 2, T/t 3, anything else 4.
__device__ __forceinline__ uint32_t base_value(uint32_t c)
{
    const uint32_t lc = c | 0x20u;
    return lc == 'a' ? 0u : lc == 'c' ? 1u : lc == 'g' ? 2u : lc == 't' ? 3u : 4u;
}

// Reverse the order of the 32 two-bit digits of v.
__device__ __forceinline__ uint64_t reverse_digits(uint64_t v)
{
    v = __builtin_bitreverse64(v);
    return ((v >> 1) & 0x5555555555555555ull) | ((v & 0x5555555555555555ull) << 1);
}

// Reverse complement of a k-mer code: complement every digit (b -> 3-b is
// b XOR 3), reverse the digit order, drop the digits above k.
__device__ __forceinline__ uint64_t revcomp(uint64_t code, uint32_t k)
{
    return reverse_digits(~code) >> (64u - 2u * k);
}

__device__ __forceinline__ uint64_t canonical(uint64_t code, uint32_t k)
{
    const uint64_t rc = revcomp(code, k);
    return code < rc ? code : rc;
}

// Bit i of x moved to bit 2i (32 -> 64 bits).
__device__ __forceinline__ uint64_t spread_bits(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// 64 consecutive bytes, one per lane, packed by the whole wave with ballots.
// fwd[]: base values as a 2-bit stream, first byte most significant
//        (byte l at bits 63-2l..62-2l of fwd[l/32], l taken mod 32);
// cmp[]: complemented base values, least significant first
//        (byte l at bits 2l..2l+1 of cmp[l/32]);
// bad:   bit l set when byte l may not be part of any window;
// start: bit l set when byte l is the first byte of a sequence.
struct Group {
    uint64_t fwd[2];
    uint64_t cmp[2];
    uint64_t bad;
    uint64_t start;
};

__device__ __forceinline__ Group pack_group(uint32_t value, bool bad, bool start)
{
    const uint64_t b0 = __ballot(!bad && (value & 1u));
    const uint64_t b1 = __ballot(!bad && (value & 2u));
    Group g;
    g.bad = __ballot(bad);
    g.start = __ballot(start);
    const uint64_t lsb0 = spread_bits((uint32_t)b0) | (spread_bits((uint32_t)b1) << 1);
    const uint64_t lsb1 = spread_bits((uint32_t)(b0 >> 32)) | (spread_bits((uint32_t)(b1 >> 32)) << 1);
    g.cmp[0] = ~lsb0;
    g.cmp[1] = ~lsb1;
    g.fwd[0] = reverse_digits(lsb0);
    g.fwd[1] = reverse_digits(lsb1);
    return g;
}

// The k-window starting at byte t (0..63) of group A, continuing into group
// B.  Returns whether it is a valid window; sets its canonical code.
__device__ __forceinline__ bool window_code(const Group &A, const Group &B, uint32_t t, uint32_t k,
                                            uint64_t kmask, uint64_t &canon)
{
    const uint32_t i = t >> 5, o = t & 31u;
    const uint64_t f0 = i ? A.fwd[1] : A.fwd[0];
    const uint64_t f1 = i ? B.fwd[0] : A.fwd[1];
    const uint64_t c0 = i ? A.cmp[1] : A.cmp[0];
    const uint64_t c1 = i ? B.cmp[0] : A.cmp[1];
    const uint64_t hi = o ? ((f0 << (2u * o)) | (f1 >> (64u - 2u * o))) : f0;
    const uint64_t lo = o ? ((c0 >> (2u * o)) | (c1 << (64u - 2u * o))) : c0;
    const uint64_t fw = hi >> (64u - 2u * k);
    const uint64_t rc = lo & kmask;
    canon = fw < rc ? fw : rc;
    const uint64_t bad = t ? ((A.bad >> t) | (B.bad << (64u - t))) : A.bad;
    const uint64_t st = t ? ((A.start >> t) | (B.start << (64u - t))) : A.start;
    const uint64_t kbits = (k >= 64u) ? ~0ull : ((1ull << k) - 1ull);
    return ((bad & kbits) == 0) && ((st & kbits & ~1ull) == 0);
}

// Largest s < n with offsets[s] <= p (0 when none); offsets has n+1 entries.
__device__ __forceinline__ uint64_t seq_of(const uint64_t *offsets, uint64_t n, uint64_t p)
{
    uint64_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (offsets[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Move s forward to the sequence that holds byte p (skipping empty ones).
__device__ __forceinline__ uint64_t seq_advance(const uint64_t *offsets, uint64_t n, uint64_t s, uint64_t p)
{
    while (s + 1 < n && offsets[s + 1] <= p)
        ++s;
    return s;
}

// Set bit (row, col) of repetition r: the bit of cell col at Bloom-filter
// position row.  OR is order-free and idempotent, so concurrent inserts need
// no ordering; the result is not used, so this is a non-returning atomic.
__device__ __forceinline__ void set_cell_bit(const Params &P, uint32_t r, uint64_t row, uint32_t col)
{
    const uint64_t bit = (row << P.S_log2) + col;
    atomicOr(P.index + (uint64_t)r * P.words_per_rep + (bit >> 5), 1u << (bit & 31u));
}

// Load L words of a row of repetition r, starting at word w0 of the row.  For
// rows narrower than a word (SW == 1, S < 32) the row is shifted down and
// masked.
template <int SW, int L>
__device__ __forceinline__ void load_row(const Params &P, uint32_t r, uint64_t row, int w0, uint32_t (&out)[L])
{
    const uint32_t *rep = P.index + (uint64_t)r * P.words_per_rep;
    if constexpr (SW == 1) {
        const uint64_t bit = row << P.S_log2;
        const uint32_t v = rep[bit >> 5];
        const uint32_t S = 1u << P.S_log2;
        out[0] = (S >= 32u) ? v : ((v >> (bit & 31u)) & ((1u << S) - 1u));
    } else if constexpr (L == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(rep + row * SW + w0);
        out[0] = v.x;
        out[1] = v.y;
    } else if constexpr (L == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(rep + row * SW + w0);
        out[0] = v.x;
        out[1] = v.y;
        out[2] = v.z;
        out[3] = v.w;
    } else {
        static_assert(L == 1, "row slice");
        out[0] = rep[row * SW + w0];
    }
}

// AND of v over the 64 lanes of the wave (every lane gets the result); call
// with the whole wave active.  DPP moves inside rows of 16 lanes (no LDS
// crossbar): the two quad swaps, then the 8- and 16-lane mirrors leave every
// lane with the AND of its row; one lane of each of the four rows finishes.
__device__ __forceinline__ uint32_t wave_and(uint32_t v)
{
    constexpr int kQuadSwap1 = 0xB1;     // quad_perm [1,0,3,2]
    constexpr int kQuadSwap2 = 0x4E;     // quad_perm [2,3,0,1]
    constexpr int kHalfMirror = 0x141;   // row_half_mirror
    constexpr int kMirror = 0x140;       // row_mirror
    v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, kQuadSwap1, 0xF, 0xF, false);
    v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, kQuadSwap2, 0xF, 0xF, false);
    v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, kHalfMirror, 0xF, 0xF, false);
    v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, kMirror, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) & (uint32_t)__builtin_amdgcn_readlane((int)v, 16) &
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) & (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

// OR of v over the 64 lanes of the wave, the same DPP pattern as wave_and.
__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
    constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap1, 0xF, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap2, 0xF, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kHalfMirror, 0xF, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kMirror, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) | (uint32_t)__builtin_amdgcn_readlane((int)v, 16) |
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) | (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

}  // namespace rambo_dev
