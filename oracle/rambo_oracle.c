/*
 * RAMBO oracle: a plain, slow, obviously correct CPU implementation of the
 * multiple-set-membership index of Gupta, Yan, Coleman, Elworth, Medini,
 * Treangen and Shrivastava, "RAMBO: Repeated And Merged BloOm Filter for
 * Ultra-fast Multiple Set Membership Testing (MSMT) on Large-Scale Data"
 * (arXiv 1910.02611).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark are the only code that may load this library.
 * It shares no code with the GPU library: every hash, encoding and table is
 * written again here from its published definition.
 *
 * Data structure (Sec. 3, Fig. 1, Alg. 1): R tables of B cells; every cell
 * is its own Bloom filter of m bits (a "BFU", Bloom filter of the union of
 * the sets the partition hash puts in that cell).  Each BFU is a separate
 * array.  Nothing is bit-sliced, blocked, fused or reordered.
 *
 * Conventions the paper leaves open (each is a reading, stated once here):
 *  - Terms are k-mers over ACGT (Sec. 5.2).  Base values A=0, C=1, G=2, T=3,
 *    case-insensitive; the first base of the window is the most significant
 *    base-4 digit.  Any other byte breaks the window.
 *  - A term is stored in canonical form: the smaller of its code and the
 *    code of its reverse complement (complement of base b is 3-b).
 *  - With ORC_FLAG_RAW_KEYS the terms are arbitrary 64-bit keys taken as
 *    they are (documents as sets and word unigrams as terms, Sec. 5.3; the
 *    caller maps a word to its key).  Such an index takes terms only: the
 *    sequence functions refuse it.
 *  - Partition hash phi_r (Alg. 1, Sec. 3.1), applied to the set identity:
 *    phi_r(i) = ((a_r * i + b_r) mod P) mod B with P = 2^61 - 1, the
 *    Carter-Wegman 2-universal family the paper cites; repetitions 0..R-1.
 *  - Bloom-filter hashes h_{r,j} (Sec. 2, Alg. 1: eta universal hash
 *    functions per filter): the multiply-shift family of Dietzfelbinger,
 *    Hagerup, Katajainen and Penttonen (J. Algorithms 1997) over a fixed
 *    bijective mix of the code, pos = floor(((a_{r,j} * mix64(x)) mod 2^64)
 *    * m / 2^64) with a_{r,j} = s_{r,j} OR 1 (odd).  mix64 is the output
 *    function of splitmix64 (Steele, Lea and Flood, OOPSLA 2014); being a
 *    bijection it keeps distinct codes distinct, and for distinct keys a
 *    random odd multiplier collides with probability at most 2/m.  For a
 *    power-of-two m this is the top log2(m) bits of the product; otherwise
 *    the floor-of-product range reduction is Lemire's (2019).  The eta
 *    multipliers of a repetition are shared by the B cells of that
 *    repetition and differ between repetitions.
 *  - Seeds: one splitmix64 stream from the master seed yields, in order,
 *    (a_r, b_r) for r = 0..R-1 with a_r = 1 + u mod (P-1), b_r = u mod P,
 *    then s_{r,j} for r = 0..R-1, j = 0..eta-1.
 *  - Answers are K-bit masks: set i is bit (i mod 32) of 32-bit word i/32.
 *  - A sequence query with no valid k-mer answers the empty set.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-22)
#define ORC_ENOMEM (-12)
#define ORC_ERANGE (-34)

#define ORC_FLAG_IDENTITY_PARTITION 1u
#define ORC_FLAG_NO_FILTERS 2u          /* parameters only: for the row scans of large indexes */
#define ORC_FLAG_RAW_KEYS 4u            /* terms are 64-bit keys, not k-mer codes */
#define ORC_NO_KMER UINT64_MAX

static const uint64_t ORC_P61 = (1ULL << 61) - 1;

/* ---------------------------------------------------------------- hashing */

/* splitmix64 output function (Steele, Lea, Flood 2014). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* splitmix64 generator step: advance the Weyl state, then mix it. */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ULL;
    return orc_mix64(*state);
}

/* Partition hash phi (Alg. 1, Sec. 3.1): ((a*i + b) mod P) mod B. */
uint32_t orc_partition_value(uint64_t a, uint64_t b, uint64_t i, uint32_t B)
{
    unsigned __int128 t = (unsigned __int128)a * i + b;
    uint64_t modp = (uint64_t)(t % ORC_P61);
    return (uint32_t)(modp % B);
}

/* Bloom-filter position (Sec. 2): multiply-shift with the odd multiplier
 * seed|1 over mix64(x), reduced to [0, m): floor((((seed|1) * mix64(x)) mod
 * 2^64) * m / 2^64). */
uint64_t orc_position(uint64_t x, uint64_t seed, uint64_t m)
{
    uint64_t h = orc_mix64(x);
    uint64_t v = (seed | 1ULL) * h; /* mod 2^64 */
    return (uint64_t)(((unsigned __int128)v * m) >> 64);
}

/* ------------------------------------------------------------- k-mer code */

static int orc_base_value(unsigned char c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

/* Code of the k bases at s: base-4 number, first base most significant.
 * Returns 1 and stores the code when all k bytes are bases, else 0. */
int orc_encode_kmer(const unsigned char *s, uint32_t k, uint64_t *code)
{
    uint64_t v = 0;
    for (uint32_t t = 0; t < k; t++) {
        int b = orc_base_value(s[t]);
        if (b < 0)
            return 0;
        v = v * 4 + (uint64_t)b;
    }
    *code = v;
    return 1;
}

/* Reverse complement: read the digits from the last base to the first,
 * replacing each base b by 3 - b. */
uint64_t orc_revcomp(uint64_t code, uint32_t k)
{
    uint64_t r = 0;
    for (uint32_t t = 0; t < k; t++) {
        uint64_t b = code & 3;
        code >>= 2;
        r = r * 4 + (3 - b);
    }
    return r;
}

uint64_t orc_canonical(uint64_t code, uint32_t k)
{
    uint64_t rc = orc_revcomp(code, k);
    return code < rc ? code : rc;
}

static int orc_code_in_range(uint64_t code, uint32_t k)
{
    return k >= 32 || code < (1ULL << (2 * k));
}

/* Canonical code of every window of every sequence.  out[offsets[s] + t] is
 * the canonical code of the window starting at base t of sequence s, or
 * ORC_NO_KMER where no valid window starts. */
void orc_extract(const uint64_t *offsets, const unsigned char *chars, uint64_t n_seqs,
                 uint32_t k, uint64_t *out)
{
    for (uint64_t s = 0; s < n_seqs; s++) {
        uint64_t beg = offsets[s], end = offsets[s + 1];
        for (uint64_t p = beg; p < end; p++) {
            uint64_t code;
            if (p + k <= end && orc_encode_kmer(chars + p, k, &code))
                out[p] = orc_canonical(code, k);
            else
                out[p] = ORC_NO_KMER;
        }
    }
}

/* ------------------------------------------------------------ the index */

typedef struct orc_index {
    uint32_t K, B, R, eta, k, flags;
    uint64_t m, seed;
    uint64_t *pa, *pb;        /* partition hash parameters, [R] */
    uint64_t *ps;             /* Bloom-filter hash seeds, [R*eta] */
    uint32_t *phi;            /* phi_r(i) at [r*K + i] */
    uint64_t *member_off;     /* SetIDs(M[b,r]): sets of cell (r,b) are */
    uint32_t *member_ids;     /*   member_ids[member_off[r*B+b] .. +1) */
    uint64_t words;           /* 64-bit words per BFU */
    uint64_t **bfu;           /* bfu[r*B + b]: the m bits of cell (r,b) */
} orc_index;

static void orc_bit_set(uint64_t *a, uint64_t p) { a[p >> 6] |= 1ULL << (p & 63); }
static int orc_bit_get(const uint64_t *a, uint64_t p) { return (int)((a[p >> 6] >> (p & 63)) & 1); }

void orc_destroy(orc_index *h)
{
    if (!h)
        return;
    if (h->bfu) {
        for (uint64_t c = 0; c < (uint64_t)h->R * h->B; c++)
            free(h->bfu[c]);   /* NULL without filters */
        free(h->bfu);
    }
    free(h->pa); free(h->pb); free(h->ps); free(h->phi);
    free(h->member_off); free(h->member_ids);
    free(h);
}

int orc_create(uint32_t K, uint32_t B, uint32_t R, uint32_t eta, uint32_t k, uint64_t m,
               uint64_t seed, uint32_t flags, orc_index **out)
{
    *out = NULL;
    if (K < 1 || B < 1 || B > K || R < 1 || eta < 1 || k < 1 || k > 32 || m < 64)
        return ORC_EINVAL;
    orc_index *h = calloc(1, sizeof *h);
    if (!h)
        return ORC_ENOMEM;
    h->K = K; h->B = B; h->R = R; h->eta = eta; h->k = k; h->m = m;
    h->seed = seed; h->flags = flags;
    h->words = (m + 63) / 64;
    h->pa = calloc(R, sizeof(uint64_t));
    h->pb = calloc(R, sizeof(uint64_t));
    h->ps = calloc((size_t)R * eta, sizeof(uint64_t));
    h->phi = calloc((size_t)R * K, sizeof(uint32_t));
    h->member_off = calloc((size_t)R * B + 1, sizeof(uint64_t));
    h->member_ids = calloc((size_t)R * K, sizeof(uint32_t));
    h->bfu = calloc((size_t)R * B, sizeof(uint64_t *));
    if (!h->pa || !h->pb || !h->ps || !h->phi || !h->member_off || !h->member_ids || !h->bfu) {
        orc_destroy(h);
        return ORC_ENOMEM;
    }

    /* Seeds, in the documented order. */
    uint64_t st = seed;
    for (uint32_t r = 0; r < R; r++) {
        h->pa[r] = 1 + orc_splitmix64_next(&st) % (ORC_P61 - 1);
        h->pb[r] = orc_splitmix64_next(&st) % ORC_P61;
    }
    for (uint32_t r = 0; r < R; r++)
        for (uint32_t j = 0; j < eta; j++)
            h->ps[(size_t)r * eta + j] = orc_splitmix64_next(&st);

    /* R independent partitions of the K sets into B cells, drawn before any
     * insertion (Alg. 1). */
    for (uint32_t r = 0; r < R; r++)
        for (uint32_t i = 0; i < K; i++)
            h->phi[(size_t)r * K + i] = (flags & ORC_FLAG_IDENTITY_PARTITION)
                                            ? i % B
                                            : orc_partition_value(h->pa[r], h->pb[r], i, B);

    /* SetIDs(M[b,r]) (Alg. 2): the sets that cell (r,b) holds, ascending. */
    uint64_t pos = 0;
    for (uint32_t r = 0; r < R; r++)
        for (uint32_t b = 0; b < B; b++) {
            h->member_off[(size_t)r * B + b] = pos;
            for (uint32_t i = 0; i < K; i++)
                if (h->phi[(size_t)r * K + i] == b)
                    h->member_ids[pos++] = i;
        }
    h->member_off[(size_t)R * B] = pos;

    /* B x R array of Bloom filters, all bits 0 (Alg. 1, Sec. 2). */
    for (uint64_t c = 0; c < (uint64_t)R * B && !(flags & ORC_FLAG_NO_FILTERS); c++) {
        h->bfu[c] = calloc(h->words, sizeof(uint64_t));
        if (!h->bfu[c]) {
            orc_destroy(h);
            return ORC_ENOMEM;
        }
    }
    *out = h;
    return ORC_OK;
}

/* Parameters, for tests: a[R], b[R], s[R*eta], phi[R*K] (any may be NULL). */
void orc_params(const orc_index *h, uint64_t *a, uint64_t *b, uint64_t *s, uint32_t *phi)
{
    if (a) memcpy(a, h->pa, h->R * sizeof(uint64_t));
    if (b) memcpy(b, h->pb, h->R * sizeof(uint64_t));
    if (s) memcpy(s, h->ps, (size_t)h->R * h->eta * sizeof(uint64_t));
    if (phi) memcpy(phi, h->phi, (size_t)h->R * h->K * sizeof(uint32_t));
}

/* Bloom-filter insert of term x into one BFU (Sec. 2): set its eta bits. */
static void orc_bf_insert(const orc_index *h, uint32_t r, uint32_t cell, uint64_t x)
{
    for (uint32_t j = 0; j < h->eta; j++)
        orc_bit_set(h->bfu[(size_t)r * h->B + cell], orc_position(x, h->ps[(size_t)r * h->eta + j], h->m));
}

/* Bloom-filter query of term x in one BFU (Sec. 2): AND of its eta bits. */
static int orc_bf_query(const orc_index *h, uint32_t r, uint32_t cell, uint64_t x)
{
    for (uint32_t j = 0; j < h->eta; j++)
        if (!orc_bit_get(h->bfu[(size_t)r * h->B + cell], orc_position(x, h->ps[(size_t)r * h->eta + j], h->m)))
            return 0;
    return 1;
}

/* The stored term of an input: the canonical k-mer of a code in [0, 4^k),
 * or the key itself in a raw-key index.  Returns 0 for a code that is not a
 * term. */
static int orc_term(const orc_index *h, uint64_t code, uint64_t *x)
{
    if (h->flags & ORC_FLAG_RAW_KEYS) {
        *x = code;
        return 1;
    }
    if (!orc_code_in_range(code, h->k))
        return 0;
    *x = orc_canonical(code, h->k);
    return 1;
}

/* Alg. 1 for one term of one set: insert it into the set's cell of every
 * repetition. */
int orc_insert_kmer(orc_index *h, uint32_t set_id, uint64_t code)
{
    if (h->flags & ORC_FLAG_NO_FILTERS)
        return ORC_EINVAL;
    if (set_id >= h->K)
        return ORC_ERANGE;
    uint64_t x;
    if (!orc_term(h, code, &x))
        return ORC_EINVAL;
    for (uint32_t r = 0; r < h->R; r++)
        orc_bf_insert(h, r, h->phi[(size_t)r * h->K + set_id], x);
    return ORC_OK;
}

/* Alg. 1 for every valid k-mer of one sequence of set set_id. */
int orc_insert_seq(orc_index *h, uint32_t set_id, const unsigned char *chars, uint64_t len)
{
    if (h->flags & ORC_FLAG_RAW_KEYS)
        return ORC_EINVAL;
    if (set_id >= h->K)
        return ORC_ERANGE;
    for (uint64_t t = 0; t + h->k <= len; t++) {
        uint64_t code;
        if (orc_encode_kmer(chars + t, h->k, &code))
            orc_insert_kmer(h, set_id, code);
    }
    return ORC_OK;
}

/* Alg. 1 over many sequences.  Threads own whole cells (r,b), so no two
 * threads write one bit array; the result is the same as the serial loop
 * because OR is order-free. */
int orc_insert_seqs(orc_index *h, const uint32_t *set_ids, const uint64_t *offsets,
                    const unsigned char *chars, uint64_t n_seqs, int nthreads)
{
    if (h->flags & (ORC_FLAG_NO_FILTERS | ORC_FLAG_RAW_KEYS))
        return ORC_EINVAL;
    for (uint64_t s = 0; s < n_seqs; s++)
        if (set_ids[s] >= h->K)
            return ORC_ERANGE;
    int64_t ncell = (int64_t)h->R * h->B;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < ncell; c++) {
        uint32_t r = (uint32_t)(c / h->B), cell = (uint32_t)(c % h->B);
        for (uint64_t s = 0; s < n_seqs; s++) {
            if (h->phi[(size_t)r * h->K + set_ids[s]] != cell)
                continue;
            for (uint64_t p = offsets[s]; p + h->k <= offsets[s + 1]; p++) {
                uint64_t code;
                if (orc_encode_kmer(chars + p, h->k, &code))
                    orc_bf_insert(h, r, cell, orc_canonical(code, h->k));
            }
        }
    }
    return ORC_OK;
}

/* Same, from k-mer codes in CSR form (codes of set set_ids[s] are
 * codes[offsets[s] .. offsets[s+1])). */
int orc_insert_kmers(orc_index *h, const uint32_t *set_ids, const uint64_t *offsets,
                     const uint64_t *codes, uint64_t n_sets, int nthreads)
{
    if (h->flags & ORC_FLAG_NO_FILTERS)
        return ORC_EINVAL;
    for (uint64_t s = 0; s < n_sets; s++) {
        if (set_ids[s] >= h->K)
            return ORC_ERANGE;
        for (uint64_t p = offsets[s]; p < offsets[s + 1]; p++) {
            uint64_t x;
            if (!orc_term(h, codes[p], &x))
                return ORC_EINVAL;
        }
    }
    int64_t ncell = (int64_t)h->R * h->B;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < ncell; c++) {
        uint32_t r = (uint32_t)(c / h->B), cell = (uint32_t)(c % h->B);
        for (uint64_t s = 0; s < n_sets; s++) {
            if (h->phi[(size_t)r * h->K + set_ids[s]] != cell)
                continue;
            for (uint64_t p = offsets[s]; p < offsets[s + 1]; p++) {
                uint64_t x = 0;
                orc_term(h, codes[p], &x);   /* every code was checked above */
                orc_bf_insert(h, r, cell, x);
            }
        }
    }
    return ORC_OK;
}

/* Alg. 2, the Bloom-filter tests: G[r*B + b] = 1 iff term x passes the BF
 * test of cell (r,b) (all 0 for a code that is not a term). */
void orc_query_cells(const orc_index *h, uint64_t code, unsigned char *G)
{
    uint64_t x;
    const int ok = orc_term(h, code, &x);
    for (uint32_t r = 0; r < h->R; r++)
        for (uint32_t b = 0; b < h->B; b++)
            G[(size_t)r * h->B + b] = (unsigned char)(ok && orc_bf_query(h, r, b, x));
}

static void orc_mask_set(uint32_t *mask, uint32_t i) { mask[i >> 5] |= 1u << (i & 31); }

/* Alg. 2 for one term: G_r = union of SetIDs(M[b,r]) over the cells b whose
 * BF holds x; A = intersection over r of G_r.  mask has ceil(K/32) words.
 * A code outside [0, 4^k) is not a term (unless the index takes raw keys)
 * and answers the empty set. */
int orc_query_kmer(const orc_index *h, uint64_t code, uint32_t *mask)
{
    if (h->flags & ORC_FLAG_NO_FILTERS)
        return ORC_EINVAL;
    uint32_t W = (h->K + 31) / 32;
    memset(mask, 0, W * sizeof(uint32_t));
    uint64_t x;
    if (!orc_term(h, code, &x))
        return ORC_EINVAL;
    unsigned char *G = malloc((size_t)h->R * h->B);
    unsigned char *inG = malloc(h->K);
    unsigned char *A = malloc(h->K);
    if (!G || !inG || !A) {
        free(G); free(inG); free(A);
        return ORC_ENOMEM;
    }
    orc_query_cells(h, code, G);
    for (uint32_t i = 0; i < h->K; i++)
        A[i] = 1;
    for (uint32_t r = 0; r < h->R; r++) {
        memset(inG, 0, h->K);
        for (uint32_t b = 0; b < h->B; b++) {
            if (!G[(size_t)r * h->B + b])
                continue;
            for (uint64_t p = h->member_off[(size_t)r * h->B + b]; p < h->member_off[(size_t)r * h->B + b + 1]; p++)
                inG[h->member_ids[p]] = 1;
        }
        for (uint32_t i = 0; i < h->K; i++)
            A[i] = A[i] & inG[i];
    }
    for (uint32_t i = 0; i < h->K; i++)
        if (A[i])
            orc_mask_set(mask, i);
    free(G); free(inG); free(A);
    return ORC_OK;
}

/* Batch of term queries; out has n * ceil(K/32) words.  Threads split the
 * queries, which only read the index. */
void orc_query_kmers(const orc_index *h, const uint64_t *codes, uint64_t n, uint32_t *out,
                     int nthreads)
{
    uint32_t W = (h->K + 31) / 32;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t q = 0; q < (int64_t)n; q++)
        orc_query_kmer(h, codes[q], out + (size_t)q * W);
}

/* Sec. 3.2.1: the answer for a sequence is the conjunction of the answers of
 * all its k-mers (the sliding window), taken literally, with no early exit.
 * Returns the number of valid k-mers; with none, the answer is empty.  A
 * raw-key index has no k-mers: every sequence answers the empty set. */
uint64_t orc_query_seq(const orc_index *h, const unsigned char *chars, uint64_t len, uint32_t *mask)
{
    uint32_t W = (h->K + 31) / 32;
    for (uint32_t w = 0; w < W; w++)
        mask[w] = 0;
    if (h->flags & ORC_FLAG_RAW_KEYS)
        return 0;
    uint32_t *one = malloc(W * sizeof(uint32_t));
    uint64_t n = 0;
    for (uint32_t i = 0; i < h->K; i++)
        orc_mask_set(mask, i);
    for (uint64_t t = 0; t + h->k <= len; t++) {
        uint64_t code;
        if (!orc_encode_kmer(chars + t, h->k, &code))
            continue;
        n++;
        orc_query_kmer(h, code, one);
        for (uint32_t w = 0; w < W; w++)
            mask[w] &= one[w];
    }
    if (n == 0)
        memset(mask, 0, W * sizeof(uint32_t));
    free(one);
    return n;
}

int orc_query_seqs(const orc_index *h, const uint64_t *offsets, const unsigned char *chars,
                   uint64_t n_reads, uint32_t *out, uint64_t *nkmers, int nthreads)
{
    if (h->flags & ORC_FLAG_RAW_KEYS)
        return ORC_EINVAL;
    uint32_t W = (h->K + 31) / 32;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < (int64_t)n_reads; q++) {
        uint64_t n = orc_query_seq(h, chars + offsets[q], offsets[q + 1] - offsets[q], out + (size_t)q * W);
        if (nkmers)
            nkmers[q] = n;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- folding */

/* Rebuild SetIDs(M[b,r]) from phi (ascending member lists). */
static void orc_build_members(orc_index *h)
{
    uint64_t pos = 0;
    for (uint32_t r = 0; r < h->R; r++)
        for (uint32_t b = 0; b < h->B; b++) {
            h->member_off[(size_t)r * h->B + b] = pos;
            for (uint32_t i = 0; i < h->K; i++)
                if (h->phi[(size_t)r * h->K + i] == b)
                    h->member_ids[pos++] = i;
        }
    h->member_off[(size_t)h->R * h->B] = pos;
}

/* Folding over (Sec. 5.2, the appendix): B -> B/2 by OR-ing the filter of
 * cell b + B/2 into the filter of cell b in every repetition; a set that was
 * in cell b + B/2 is now in cell b, so phi becomes phi mod (B/2).  B must be
 * even. */
int orc_fold(orc_index *h)
{
    if (h->B % 2 != 0 || (h->flags & ORC_FLAG_NO_FILTERS))
        return ORC_EINVAL;
    uint32_t half = h->B / 2;
    uint64_t **bfu = calloc((size_t)h->R * half, sizeof(uint64_t *));
    if (!bfu)
        return ORC_ENOMEM;
    for (uint32_t r = 0; r < h->R; r++)
        for (uint32_t b = 0; b < half; b++) {
            uint64_t *lo = h->bfu[(size_t)r * h->B + b], *hi = h->bfu[(size_t)r * h->B + b + half];
            for (uint64_t w = 0; w < h->words; w++)
                lo[w] |= hi[w];
            free(hi);
            bfu[(size_t)r * half + b] = lo;
        }
    free(h->bfu);
    h->bfu = bfu;
    h->B = half;
    for (uint64_t t = 0; t < (uint64_t)h->R * h->K; t++)
        h->phi[t] %= half;
    orc_build_members(h);
    return ORC_OK;
}

/* Replace the partition by phi[r*K + i] < B (test hook: an index built
 * directly with a given partition).  Only on an empty index. */
int orc_set_partition(orc_index *h, const uint32_t *phi)
{
    for (uint64_t t = 0; t < (uint64_t)h->R * h->K; t++)
        if (phi[t] >= h->B)
            return ORC_EINVAL;
    memcpy(h->phi, phi, (size_t)h->R * h->K * sizeof(uint32_t));
    orc_build_members(h);
    return ORC_OK;
}

/* ------------------------------------------------- rows of large indexes */

/* Index sizes beyond host memory are checked through rows: row p of
 * repetition r is the B-bit vector whose bit b is bit p of BFU(r,b).  A row is
 * computed from its definition (Alg. 1): bit b is set iff some term x of some
 * set i with phi_r(i) = b has pos_{r,j}(x) = p for some j.  Rows are stored
 * as BW = ceil(B/64) words, bit b at word b/64, bit b%64.  A row key is
 * r*m + p. */

static uint64_t orc_row_words(const orc_index *h) { return (h->B + 63) / 64; }

static void orc_atomic_or64(uint64_t *w, uint64_t v)
{
    __atomic_fetch_or(w, v, __ATOMIC_RELAXED);
}

/* Index of key in the ascending array keys[0..n), or n if absent. */
static uint64_t orc_find_key(const uint64_t *keys, uint64_t n, uint64_t key)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && keys[lo] == key ? lo : n;
}

/* One pass over every window of every sequence (sequence s belongs to set
 * set_ids[s]).  Keeps (a) with D > 0, every row p with p % D == 0:
 * sampled[((r*(m/D)) + p/D) * BW ...]; (b) the rows whose keys are listed
 * in keys[0..n_keys) (ascending, distinct): rows[t*BW ...].  Threads take
 * whole sequences and OR bits with atomic ORs (OR is order-free).  The
 * arrays must be zeroed by the caller.  m must be a multiple of D. */
int orc_scan_rows(const orc_index *h, const uint32_t *set_ids, const uint64_t *offsets,
                  const unsigned char *chars, uint64_t n_seqs, uint64_t D, uint64_t *sampled,
                  const uint64_t *keys, uint64_t n_keys, uint64_t *rows, int nthreads, int progress)
{
    uint64_t done = 0;   /* sequences finished, for the progress lines */
    if ((D > 0 && h->m % D != 0) || (h->flags & ORC_FLAG_RAW_KEYS))
        return ORC_EINVAL;
    for (uint64_t s = 0; s < n_seqs; s++)
        if (set_ids[s] >= h->K)
            return ORC_ERANGE;
    const uint64_t BW = orc_row_words(h);
    /* which positions are asked for: one bit per (r, p), behind a small
     * cache-resident bitmap of the keys' low bits that turns most misses
     * away before the large one is touched */
    const uint64_t small_bits = 1ULL << 30;
    uint64_t *want = NULL, *want_small = NULL;
    if (n_keys > 0) {
        want = calloc(((uint64_t)h->R * h->m + 63) / 64, sizeof(uint64_t));
        want_small = calloc(small_bits / 64, sizeof(uint64_t));
        if (!want || !want_small) {
            free(want);
            free(want_small);
            return ORC_ENOMEM;
        }
        for (uint64_t t = 0; t < n_keys; t++) {
            orc_bit_set(want, keys[t]);
            orc_bit_set(want_small, keys[t] & (small_bits - 1));
        }
    }
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t s = 0; s < (int64_t)n_seqs; s++) {
        uint32_t set = set_ids[s];
        for (uint64_t p = offsets[s]; p + h->k <= offsets[s + 1]; p++) {
            uint64_t code;
            if (!orc_encode_kmer(chars + p, h->k, &code))
                continue;
            uint64_t x = orc_canonical(code, h->k);
            for (uint32_t r = 0; r < h->R; r++) {
                uint32_t b = h->phi[(size_t)r * h->K + set];
                uint64_t bit = 1ULL << (b & 63);
                for (uint32_t j = 0; j < h->eta; j++) {
                    uint64_t pos = orc_position(x, h->ps[(size_t)r * h->eta + j], h->m);
                    if (D > 0 && pos % D == 0)
                        orc_atomic_or64(&sampled[((uint64_t)r * (h->m / D) + pos / D) * BW + b / 64], bit);
                    uint64_t key = (uint64_t)r * h->m + pos;
                    if (want && orc_bit_get(want_small, key & (small_bits - 1)) && orc_bit_get(want, key)) {
                        uint64_t t = orc_find_key(keys, n_keys, key);
                        orc_atomic_or64(&rows[t * BW + b / 64], bit);
                    }
                }
            }
        }
        if (progress) {
            uint64_t d = __atomic_add_fetch(&done, 1, __ATOMIC_RELAXED);
            if (d * 20 / n_seqs != (d - 1) * 20 / n_seqs) {
                fprintf(stderr, "orc_scan_rows: %llu of %llu sequences\n", (unsigned long long)d,
                        (unsigned long long)n_seqs);
                fflush(stderr);
            }
        }
    }
    free(want);
    free(want_small);
    return ORC_OK;
}

/* The BFU of one cell (r, b) of an index too large for host memory (Alg. 1
 * restricted to that cell): every valid window of every given sequence
 * whose set the partition hash puts in cell b of repetition r sets bits
 * pos_{r,j}(x), j < eta; sequences of other cells are passed over.  out:
 * ceil(m/64) words, OR-ed into (the caller clears it), bit p of word p/64. */
int orc_cell_bits(const orc_index *h, uint32_t r, uint32_t b, const uint32_t *set_ids, const uint64_t *offsets,
                  const unsigned char *chars, uint64_t n_seqs, uint64_t *out, int nthreads)
{
    if (r >= h->R || b >= h->B || (h->flags & ORC_FLAG_RAW_KEYS))
        return ORC_EINVAL;
    for (uint64_t s = 0; s < n_seqs; s++)
        if (set_ids[s] >= h->K)
            return ORC_ERANGE;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t s = 0; s < (int64_t)n_seqs; s++) {
        if (h->phi[(size_t)r * h->K + set_ids[s]] != b)
            continue;
        for (uint64_t p = offsets[s]; p + h->k <= offsets[s + 1]; p++) {
            uint64_t code;
            if (!orc_encode_kmer(chars + p, h->k, &code))
                continue;
            uint64_t x = orc_canonical(code, h->k);
            for (uint32_t j = 0; j < h->eta; j++) {
                uint64_t pos = orc_position(x, h->ps[(size_t)r * h->eta + j], h->m);
                orc_atomic_or64(&out[pos / 64], 1ULL << (pos % 64));
            }
        }
    }
    (void)nthreads;
    return ORC_OK;
}

/* Keys r*m + pos_{r,j}(x) of every valid window of every read, in window
 * order (R*eta per window); returns how many there are (at most cap are
 * written). */
uint64_t orc_window_keys(const orc_index *h, const uint64_t *offsets, const unsigned char *chars,
                         uint64_t n_reads, uint64_t *out, uint64_t cap)
{
    uint64_t n = 0;
    for (uint64_t q = 0; q < n_reads; q++)
        for (uint64_t p = offsets[q]; p + h->k <= offsets[q + 1]; p++) {
            uint64_t code;
            if (!orc_encode_kmer(chars + p, h->k, &code))
                continue;
            uint64_t x = orc_canonical(code, h->k);
            for (uint32_t r = 0; r < h->R; r++)
                for (uint32_t j = 0; j < h->eta; j++) {
                    if (n < cap)
                        out[n] = (uint64_t)r * h->m + orc_position(x, h->ps[(size_t)r * h->eta + j], h->m);
                    n++;
                }
        }
    return n;
}

/* Alg. 2 for one term with its Bloom-filter bits read from rows (keys and
 * rows as orc_scan_rows leaves them): cell (r,b) passes iff bit b of every
 * row r*m + pos_{r,j}(x) is set; A = intersection over r of the union of
 * SetIDs(M[b,r]) over the passing cells.  mask: ceil(K/32) words.  inG and
 * A are K-byte work arrays. */
static int orc_query_kmer_rows(const orc_index *h, uint64_t x, const uint64_t *keys, uint64_t n_keys,
                               const uint64_t *rows, uint32_t *mask, unsigned char *inG, unsigned char *A)
{
    const uint64_t BW = orc_row_words(h);
    uint32_t W = (h->K + 31) / 32;
    memset(mask, 0, W * sizeof(uint32_t));
    for (uint32_t i = 0; i < h->K; i++)
        A[i] = 1;
    for (uint32_t r = 0; r < h->R; r++) {
        /* the eta rows of x in repetition r (each holds bit pos_{r,j}(x) of
         * every cell) */
        const uint64_t *row[64];
        if (h->eta > 64)
            return ORC_EINVAL;
        for (uint32_t j = 0; j < h->eta; j++) {
            uint64_t key = (uint64_t)r * h->m + orc_position(x, h->ps[(size_t)r * h->eta + j], h->m);
            uint64_t t = orc_find_key(keys, n_keys, key);
            if (t == n_keys)
                return ORC_EINVAL;
            row[j] = rows + t * BW;
        }
        memset(inG, 0, h->K);
        for (uint32_t b = 0; b < h->B; b++) {
            int pass = 1;
            for (uint32_t j = 0; j < h->eta && pass; j++)
                pass = (int)((row[j][b / 64] >> (b & 63)) & 1);
            if (!pass)
                continue;
            for (uint64_t p = h->member_off[(size_t)r * h->B + b]; p < h->member_off[(size_t)r * h->B + b + 1]; p++)
                inG[h->member_ids[p]] = 1;
        }
        for (uint32_t i = 0; i < h->K; i++)
            A[i] = A[i] & inG[i];
    }
    for (uint32_t i = 0; i < h->K; i++)
        if (A[i])
            orc_mask_set(mask, i);
    return ORC_OK;
}

/* Sec. 3.2.1 for reads, from rows: the conjunction of the answers of all
 * valid windows, literally as orc_query_seq; empty when a read has none.
 * Returns ORC_EINVAL if some needed row was not provided. */
int orc_query_seqs_rows(const orc_index *h, const uint64_t *offsets, const unsigned char *chars,
                        uint64_t n_reads, const uint64_t *keys, uint64_t n_keys, const uint64_t *rows,
                        uint32_t *out, uint64_t *nkmers, int nthreads)
{
    if (h->flags & ORC_FLAG_RAW_KEYS)
        return ORC_EINVAL;
    uint32_t W = (h->K + 31) / 32;
    int rc = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < (int64_t)n_reads; q++) {
        uint32_t *mask = out + (size_t)q * W;
        uint32_t *one = malloc(W * sizeof(uint32_t));
        unsigned char *inG = malloc(h->K), *A = malloc(h->K);
        uint64_t n = 0;
        if (!one || !inG || !A) {
            __atomic_store_n(&rc, ORC_ENOMEM, __ATOMIC_RELAXED);
        } else {
            for (uint32_t w = 0; w < W; w++)
                mask[w] = 0;
            for (uint32_t i = 0; i < h->K; i++)
                orc_mask_set(mask, i);
            for (uint64_t p = offsets[q]; p + h->k <= offsets[q + 1]; p++) {
                uint64_t code;
                if (!orc_encode_kmer(chars + p, h->k, &code))
                    continue;
                n++;
                if (orc_query_kmer_rows(h, orc_canonical(code, h->k), keys, n_keys, rows, one, inG, A) != ORC_OK) {
                    __atomic_store_n(&rc, ORC_EINVAL, __ATOMIC_RELAXED);
                    break;
                }
                for (uint32_t w = 0; w < W; w++)
                    mask[w] &= one[w];
            }
            if (n == 0)
                memset(mask, 0, W * sizeof(uint32_t));
        }
        if (nkmers)
            nkmers[q] = n;
        free(one); free(inG); free(A);
    }
    return rc;
}

/* ------------------------------------------------------------ inspection */

/* Number of 1 bits in every BFU, [R*B]. */
void orc_fill_counts(const orc_index *h, uint64_t *out)
{
    for (uint64_t c = 0; c < (uint64_t)h->R * h->B; c++) {
        uint64_t n = 0;
        for (uint64_t w = 0; w < h->words; w++)
            n += (uint64_t)__builtin_popcountll(h->bfu[c][w]);
        out[c] = n;
    }
}

/* The raw bits of BFU (r,b): ceil(m/64) words, bit p at word p/64, bit p%64. */
void orc_copy_bfu(const orc_index *h, uint32_t r, uint32_t b, uint64_t *out)
{
    memcpy(out, h->bfu[(size_t)r * h->B + b], h->words * sizeof(uint64_t));
}

/* Bit p of every BFU of repetition r, for a list of positions:
 * out[t*B + b] = bit rows[t] of cell (r,b). */
void orc_bits_at(const orc_index *h, uint32_t r, const uint64_t *rows, uint64_t n, unsigned char *out)
{
    for (uint64_t t = 0; t < n; t++)
        for (uint32_t b = 0; b < h->B; b++)
            out[t * h->B + b] = (unsigned char)orc_bit_get(h->bfu[(size_t)r * h->B + b], rows[t]);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
