/*
 * Drives every entry point of the oracle on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py).
 * Exits 0 when the few invariants checked here hold; the sanitizers abort
 * on any out-of-bounds access, leak or undefined operation.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_index orc_index;
uint64_t orc_mix64(uint64_t z);
uint64_t orc_splitmix64_next(uint64_t *state);
uint32_t orc_partition_value(uint64_t a, uint64_t b, uint64_t i, uint32_t B);
uint64_t orc_position(uint64_t x, uint64_t seed, uint64_t m);
int orc_encode_kmer(const unsigned char *s, uint32_t k, uint64_t *code);
uint64_t orc_canonical(uint64_t code, uint32_t k);
void orc_extract(const uint64_t *offsets, const unsigned char *chars, uint64_t n_seqs, uint32_t k, uint64_t *out);
int orc_create(uint32_t K, uint32_t B, uint32_t R, uint32_t eta, uint32_t k, uint64_t m, uint64_t seed,
               uint32_t flags, orc_index **out);
void orc_destroy(orc_index *h);
void orc_params(const orc_index *h, uint64_t *a, uint64_t *b, uint64_t *s, uint32_t *phi);
int orc_insert_seqs(orc_index *h, const uint32_t *set_ids, const uint64_t *offsets, const unsigned char *chars,
                    uint64_t n_seqs, int nthreads);
int orc_insert_kmers(orc_index *h, const uint32_t *set_ids, const uint64_t *offsets, const uint64_t *codes,
                     uint64_t n_sets, int nthreads);
void orc_query_kmers(const orc_index *h, const uint64_t *codes, uint64_t n, uint32_t *out, int nthreads);
int orc_query_seqs(const orc_index *h, const uint64_t *offsets, const unsigned char *chars, uint64_t n_reads,
                   uint32_t *out, uint64_t *nkmers, int nthreads);
int orc_fold(orc_index *h);
int orc_scan_rows(const orc_index *h, const uint32_t *set_ids, const uint64_t *offsets, const unsigned char *chars,
                  uint64_t n_seqs, uint64_t D, uint64_t *sampled, const uint64_t *keys, uint64_t n_keys,
                  uint64_t *rows, int nthreads, int progress);
int orc_cell_bits(const orc_index *h, uint32_t r, uint32_t b, const uint32_t *set_ids, const uint64_t *offsets,
                  const unsigned char *chars, uint64_t n_seqs, uint64_t *out, int nthreads);
uint64_t orc_window_keys(const orc_index *h, const uint64_t *offsets, const unsigned char *chars,
                         uint64_t n_reads, uint64_t *out, uint64_t cap);
int orc_query_seqs_rows(const orc_index *h, const uint64_t *offsets, const unsigned char *chars, uint64_t n_reads,
                        const uint64_t *keys, uint64_t n_keys, const uint64_t *rows, uint32_t *out,
                        uint64_t *nkmers, int nthreads);
void orc_fill_counts(const orc_index *h, uint64_t *out);
void orc_copy_bfu(const orc_index *h, uint32_t r, uint32_t b, uint64_t *out);
void orc_bits_at(const orc_index *h, uint32_t r, const uint64_t *rows, uint64_t n, unsigned char *out);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

int main(void)
{
    enum { K = 40, B = 8, R = 3, ETA = 2, KMER = 21, LEN = 600 };
    const uint64_t m = 1 << 12;
    const char *alpha = "ACGTacgtN";
    uint64_t st = 12345;
    /* K sequences of LEN bytes (a few N and lower-case bases), one per set */
    unsigned char *chars = malloc(K * LEN);
    uint64_t offsets[K + 1];
    uint32_t ids[K];
    for (int s = 0; s < K; s++) {
        offsets[s] = (uint64_t)s * LEN;
        ids[s] = (uint32_t)s;
        for (int p = 0; p < LEN; p++) {
            uint64_t u = orc_splitmix64_next(&st);
            chars[s * LEN + p] = (unsigned char)alpha[(u % 100) < 2 ? 8 : u % 8];
        }
    }
    offsets[K] = (uint64_t)K * LEN;

    orc_index *h = NULL, *lean = NULL;
    CHECK(orc_create(K, B, R, ETA, KMER, m, 7, 0, &h) == 0);
    CHECK(orc_create(K, B, R, ETA, KMER, m, 7, 2, &lean) == 0);
    CHECK(orc_insert_seqs(h, ids, offsets, chars, K, 1) == 0);

    /* every set's own sequence is in its answer (no false negatives) */
    uint32_t W = (K + 31) / 32;
    uint32_t *masks = calloc((size_t)K * W, 4);
    uint64_t *nk = calloc(K, 8);
    CHECK(orc_query_seqs(h, offsets, chars, K, masks, nk, 1) == 0);
    for (int s = 0; s < K; s++)
        CHECK(nk[s] == 0 || (masks[s * W + s / 32] >> (s % 32) & 1));

    /* codes of every window, then the k-mer queries */
    uint64_t *codes = malloc(K * LEN * 8);
    orc_extract(offsets, chars, K, KMER, codes);
    uint32_t *km = calloc((size_t)K * LEN * W, 4);
    orc_query_kmers(h, codes, (uint64_t)K * LEN, km, 1);

    /* rows of the lean index against the filters */
    uint64_t nkeys = orc_window_keys(lean, offsets, chars, 4, NULL, 0);
    uint64_t *keys = malloc((nkeys + 1) * 8);
    CHECK(orc_window_keys(lean, offsets, chars, 4, keys, nkeys) == nkeys);
    qsort(keys, nkeys, 8, cmp_u64);
    uint64_t u = 0;
    for (uint64_t i = 0; i < nkeys; i++)
        if (i == 0 || keys[i] != keys[u - 1])
            keys[u++] = keys[i];
    uint64_t BW = (B + 63) / 64;
    uint64_t *rows = calloc(u * BW + 1, 8), *sampled = calloc(R * (m / 16) * BW, 8);
    CHECK(orc_scan_rows(lean, ids, offsets, chars, K, 16, sampled, keys, u, rows, 1, 0) == 0);
    uint32_t *m2 = calloc(4 * W, 4);
    uint64_t nk2[4];
    CHECK(orc_query_seqs_rows(lean, offsets, chars, 4, keys, u, rows, m2, nk2, 1) == 0);
    CHECK(memcmp(m2, masks, 4 * W * 4) == 0);
    uint64_t *cell = calloc(m / 64, 8), *bfu = calloc(m / 64, 8);
    CHECK(orc_cell_bits(lean, 1, 3, ids, offsets, chars, K, cell, 1) == 0);
    orc_copy_bfu(h, 1, 3, bfu);
    CHECK(memcmp(cell, bfu, m / 8) == 0);
    uint64_t fills[R * B];
    orc_fill_counts(h, fills);
    uint64_t probe[3] = {0, 5, m - 1};
    unsigned char bits[3 * B];
    orc_bits_at(h, 2, probe, 3, bits);

    /* raw keys, then folding over */
    orc_index *raw = NULL;
    CHECK(orc_create(K, B, R, ETA, KMER, m, 9, 4, &raw) == 0);
    uint64_t koff[K + 1];
    for (int s = 0; s <= K; s++)
        koff[s] = (uint64_t)s * 10;
    uint64_t *rk = malloc(K * 10 * 8);
    for (int i = 0; i < K * 10; i++)
        rk[i] = orc_mix64((uint64_t)i);
    CHECK(orc_insert_kmers(raw, ids, koff, rk, K, 1) == 0);
    CHECK(orc_fold(h) == 0);
    CHECK(orc_query_seqs(h, offsets, chars, K, masks, nk, 1) == 0);
    for (int s = 0; s < K; s++)
        CHECK(nk[s] == 0 || (masks[s * W + s / 32] >> (s % 32) & 1));

    orc_destroy(h);
    orc_destroy(lean);
    orc_destroy(raw);
    free(chars); free(masks); free(nk); free(codes); free(km); free(keys); free(rows); free(sampled);
    free(m2); free(cell); free(bfu); free(rk);
    printf("oracle sanitizer run ok\n");
    return 0;
}
