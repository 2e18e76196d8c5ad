/*
 * rambo.h - C ABI of the MI355X (gfx950) RAMBO index.
 *
 * RAMBO (Repeated And Merged BloOm Filter, Gupta et al., arXiv 1910.02611)
 * answers multiple-set-membership queries (Sec. 1): given K sets of terms
 * and a query term q, return the sets that hold q.  The K sets are split by
 * R independent partition hashes into B cells each (Sec. 3, Fig. 1); every
 * cell is one Bloom filter of m bits over the union of its sets (a "BFU").
 * Insertion is Alg. 1, a term query is Alg. 2 (union over positive cells,
 * intersection over repetitions), a sequence query is the conjunction over
 * all of its k-mers (Sec. 3.2.1).
 *
 * Terms are k-mers (Sec. 5.2), stored canonically: the smaller of the code
 * and the code of the reverse complement, where a code packs A=0 C=1 G=2
 * T=3 into base-4 digits with the first base most significant.  Bytes other
 * than ACGTacgt break the k-window.
 *
 * Hashes (the paper fixes only their kind; these are this library's choice,
 * fixed so that two implementations agree bit for bit):
 *   splitmix64 stream from cfg.seed (Steele, Lea, Flood 2014): for r = 0..R-1
 *   draw a_r = 1 + u mod (2^61-2), b_r = u mod (2^61-1); then for r, j draw
 *   s_{r,j}.  phi_r(i) = ((a_r i + b_r) mod (2^61-1)) mod B (Carter-Wegman,
 *   the 2-universal family of Sec. 3.1).  Position j of term x in repetition
 *   r: multiply-shift (Dietzfelbinger et al. 1997) with the odd multiplier
 *   a_{r,j} = s_{r,j} | 1 over mix64(x), splitmix64's output function (a
 *   bijection): floor(((a_{r,j} * mix64(x)) mod 2^64) * m / 2^64); the B
 *   cells of one repetition share these positions.
 *
 * Index layout in device memory (bit-sliced): repetition r is a block of
 * words_per_rep 32-bit words; inside it, row p (a Bloom-filter position)
 * holds the bits of all B cells at that position: bit p*S + b of the block
 * (word (p*S+b)/32, bit (p*S+b)%32) is bit p of cell b, where the row
 * stride S = max(8, next power of two >= B).  One row read therefore
 * returns position p of every cell of the repetition.
 *
 * Answers: a K-bit mask per query, W = ceil(K/32) uint32 words; set i is bit
 * i%32 of word i/32; bits >= K are 0.
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers owned by the caller; they must stay
 *    valid until the work on `stream` has finished.  Sizes are host values.
 *  - Calls are asynchronous and ordered on `stream` (0 = the null stream).
 *    One handle serves one host thread at a time.  The handle's own device
 *    scratch (the partitioned insert's slabs, the per-read state of batched
 *    read queries) is shared by its calls whatever their stream: a call that
 *    uses it on a stream other than the previous user's first waits for
 *    that user's work, so calls on different streams never share it at
 *    once.  The index itself is the caller's to order: an insert and a query
 *    on two streams with no dependency between them may see each other's
 *    bits or not.  Scratch that a captured graph may still replay on is
 *    kept until rambo_destroy when a later call grows it.
 *  - Return 0 on success or a negative RAMBO_E* code.  Errors found on the
 *    host return at once and enqueue nothing.  Errors found on the device
 *    (a set id >= K, a code >= 4^k) skip the item (insert) or give it an
 *    empty answer (query) and set a sticky flag that rambo_sync_status()
 *    reports and clears.
 */
#ifndef RAMBO_H
#define RAMBO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAMBO_OK 0
#define RAMBO_EINVAL (-22)     /* bad configuration or argument */
#define RAMBO_ENOMEM (-12)     /* device allocation failed */
#define RAMBO_ERANGE (-34)     /* a set id >= K was seen on the device */
#define RAMBO_EOVERFLOW (-75)  /* output capacity too small */
#define RAMBO_EHIP (-1000)     /* HIP runtime error; see rambo_last_error */
#define RAMBO_ECODE (-1001)    /* a k-mer code >= 4^k was seen on the device */
#define RAMBO_EIO (-5)         /* file could not be opened, read or written */

/* Test hook: phi_r(i) = i mod B for every r (with B = K and R = 1 the index
 * is a plain array of Bloom filters, the special case of Sec. 4.3). */
#define RAMBO_FLAG_IDENTITY_PARTITION 1u

/* Terms are arbitrary 64-bit keys taken as they are, with no canonical
 * k-mer form and no range check: documents as sets and word unigrams as
 * terms (Sec. 5.3; mapping a word to its key is the caller's).  Such an
 * index takes keys through rambo_insert_kmers and rambo_query_kmers, whose
 * "codes" are then the keys; k is unused, and every entry point that takes
 * sequences (insert_seqs, query_seqs, query_seqs_ids, extract_kmers, the
 * plain sequence path and the query server) returns RAMBO_EINVAL. */
#define RAMBO_FLAG_RAW_KEYS 4u

/* Limits of this implementation. */
#define RAMBO_MAX_B 4096u
#define RAMBO_MAX_R 16u
#define RAMBO_MAX_RETA 32u     /* R * eta */

typedef struct rambo_config {
    uint32_t K;      /* number of sets, >= 1 */
    uint32_t B;      /* cells per repetition, 1 <= B <= min(K, RAMBO_MAX_B) */
    uint32_t R;      /* repetitions, 1 <= R <= RAMBO_MAX_R */
    uint32_t eta;    /* Bloom-filter hashes per repetition, R*eta <= RAMBO_MAX_RETA */
    uint32_t k;      /* k-mer length, 1 <= k <= 32 */
    uint32_t flags;  /* RAMBO_FLAG_* */
    uint64_t m;      /* bits per Bloom filter (positions per repetition), >= 64 */
    uint64_t seed;   /* master seed of all hash functions */
} rambo_config;

typedef struct rambo_info {
    uint32_t row_bits;       /* S, the row stride in bits */
    uint32_t mask_words;     /* W = ceil(K/32) */
    uint64_t words_per_rep;  /* 32-bit words per repetition block */
    uint64_t index_bytes;    /* R * words_per_rep * 4 */
    const uint32_t *index;   /* device pointer to the index (owned by the handle) */
} rambo_info;

typedef struct rambo rambo_t;

/* Create an index: validate cfg, derive the seeds, build phi_r and the cell
 * membership tables on the device (SetIDs(M[b,r]) of Alg. 2), allocate and
 * zero the R*B Bloom filters (the set-up of Alg. 1).  Synchronous.
 * Returns RAMBO_EINVAL for a bad cfg, RAMBO_ENOMEM, RAMBO_EHIP. */
int rambo_create(const rambo_config *cfg, rambo_t **out);

/* Free the index and every buffer of the handle after synchronising the
 * device.  NULL is a no-op. */
void rambo_destroy(rambo_t *h);

/* Alg. 1 from k-mer codes.  Set set_ids[s] (s < n_sets) receives the codes
 * codes[offsets[s] .. offsets[s+1]); offsets has n_sets+1 entries,
 * non-decreasing, with offsets[n_sets] <= n_codes.  Codes need not be
 * canonical.  Repeated calls OR into the same index (streaming updates,
 * Sec. 3.1); order does not matter.  Device errors: RAMBO_ERANGE (set id),
 * RAMBO_ECODE (code >= 4^k, k-mer indexes only) - the item is skipped.
 * With RAMBO_FLAG_RAW_KEYS the codes are the keys.  The insert policy
 * (rambo_set_insert_policy) applies as for sequences. */
int rambo_insert_kmers(rambo_t *h, const uint32_t *set_ids, const uint64_t *offsets,
                       uint64_t n_sets, const uint64_t *codes, uint64_t n_codes,
                       hipStream_t stream);

/* Alg. 1 from sequences: every valid k-window of sequence s (bytes
 * chars[offsets[s] .. offsets[s+1])) is inserted into set set_ids[s].
 * Windows never span two sequences.  offsets: n_seqs+1 entries,
 * non-decreasing, offsets[n_seqs] <= n_chars. */
int rambo_insert_seqs(rambo_t *h, const uint32_t *set_ids, const uint64_t *offsets,
                      uint64_t n_seqs, const uint8_t *chars, uint64_t n_chars,
                      hipStream_t stream);

/* Alg. 2 for n k-mer codes: out_masks[q*W .. q*W+W) receives the answer of
 * codes[q].  A code >= 4^k gets an empty mask (and RAMBO_ECODE); with
 * RAMBO_FLAG_RAW_KEYS every 64-bit code is a key. */
int rambo_query_kmers(rambo_t *h, const uint64_t *codes, uint64_t n,
                      uint32_t *out_masks, hipStream_t stream);

/* Sec. 3.2.1 for n_sets sets of terms given as codes (or raw keys with
 * RAMBO_FLAG_RAW_KEYS): term set q is codes[offsets[q] .. offsets[q+1]) and
 * its answer, out_masks[q*W .. q*W+W), is the intersection of the answers
 * of its terms (Alg. 2 per term) - for a document index, the documents that
 * hold every word of a multi-word query.  offsets: n_sets+1 device entries,
 * non-decreasing, offsets[n_sets] <= n_codes.  An empty term set answers the
 * empty set.  A code >= 4^k (k-mer indexes) empties its set's answer and
 * raises RAMBO_ECODE.  codes may be NULL when n_codes is 0. */
int rambo_query_termsets(rambo_t *h, const uint64_t *offsets, uint64_t n_sets,
                         const uint64_t *codes, uint64_t n_codes, uint32_t *out_masks,
                         hipStream_t stream);

/* Sec. 3.2.1 for n_reads sequences (bytes chars[offsets[q] .. offsets[q+1])):
 * the answer is the intersection of the answers of all valid k-windows of
 * the read.  A read with no valid window answers the empty set.
 * out_masks: n_reads*W words.  out_nkmers (may be NULL): number of valid
 * windows of each read. */
int rambo_query_seqs(rambo_t *h, const uint64_t *offsets, uint64_t n_reads,
                     const uint8_t *chars, uint64_t n_chars, uint32_t *out_masks,
                     uint32_t *out_nkmers, hipStream_t stream);

/* The answers of rambo_query_seqs as ascending set-ID lists (Sec. 3.2.1; the
 * compacted form of the K-bit mask, for large K where most answers are
 * short).  id_offsets (n_reads+1 uint64) receives the list boundaries: read
 * q's IDs are ids[id_offsets[q] .. id_offsets[q+1]), and id_offsets[n_reads]
 * is the total needed.  ids holds cap uint32 entries (may be NULL when cap is
 * 0).  id_offsets is always written in full; a read whose list would end
 * beyond cap gets no IDs written, and the call then raises the sticky
 * RAMBO_EOVERFLOW status (reported by rambo_sync_status), after which the
 * caller may call again with cap >= id_offsets[n_reads].  out_nkmers as in
 * rambo_query_seqs.  Uses the same per-read state as the work-queue form. */
int rambo_query_seqs_ids(rambo_t *h, const uint64_t *offsets, uint64_t n_reads,
                         const uint8_t *chars, uint64_t n_chars, uint64_t *id_offsets,
                         uint32_t *ids, uint64_t cap, uint32_t *out_nkmers, hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rambo_query_seqs_ids with its per-read state and scan totals in a
 * fixed array of RAMBO_NOALLOC_SCRATCH_BYTES per GPU, reserved when the
 * library's code is loaded on that GPU and held until the process ends.
 * Arguments, answers, overflow and errors as in rambo_query_seqs_ids; the
 * call allocates nothing.  A batch larger than the array holds (more than
 * rambo_query_seqs_ids_noalloc_max_reads(h) reads; about 4*(R*S/32+5)
 * bytes per read) is refused with RAMBO_EINVAL before any work is queued.
 * Every call on one GPU, from any handle, uses the same array, which keeps
 * the last call's contents (each call sets up what it reads): calls whose
 * work may overlap on the GPU (different streams with no dependency, or
 * several host threads) race on it and give wrong answers, so order them
 * on one stream or with events.  RAMBO_EHIP if the array's device address
 * could not be found when the handle was created (rambo_last_error says
 * why). */
#define RAMBO_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rambo_query_seqs_ids_noalloc(rambo_t *h, const uint64_t *offsets, uint64_t n_reads,
                                 const uint8_t *chars, uint64_t n_chars, uint64_t *id_offsets,
                                 uint32_t *ids, uint64_t cap, uint32_t *out_nkmers,
                                 hipStream_t stream);
uint64_t rambo_query_seqs_ids_noalloc_max_reads(const rambo_t *h);

/* ---- support ---------------------------------------------------------- */

/* Canonical code of the k-window starting at every byte (the term
 * extraction of Sec. 3.2.1 / Sec. 5.2): out_codes[p] for p < n_chars, or
 * UINT64_MAX where no valid window of the same sequence starts at p. */
int rambo_extract_kmers(rambo_t *h, const uint64_t *offsets, uint64_t n_seqs,
                        const uint8_t *chars, uint64_t n_chars, uint64_t *out_codes,
                        hipStream_t stream);

/* The "plain" path: the same answers as rambo_query_kmers /
 * rambo_query_seqs, computed by one kernel launch per query. */
int rambo_query_kmers_plain(rambo_t *h, const uint64_t *codes, uint64_t n,
                            uint32_t *out_masks, hipStream_t stream);
int rambo_query_seqs_plain(rambo_t *h, const uint64_t *offsets, uint64_t n_reads,
                           const uint8_t *chars, uint64_t n_chars, uint32_t *out_masks,
                           uint32_t *out_nkmers, hipStream_t stream);

/* How rambo_insert_seqs and rambo_insert_kmers apply bits (the result is
 * the same either way):
 * DIRECT issues one atomicOr per bit target (Alg. 1 as written); PARTITIONED
 * sorts the targets by address into regions of the index and ORs each region
 * in on-chip memory, which avoids the device's atomic-rate limit on bulk
 * inserts; AUTO picks by the number of targets.  scratch_bytes caps the
 * device scratch of the partitioned path (0 = 95% of the free memory left
 * after keeping 8 GiB free, at most 192 GiB; the scratch takes about 8.5
 * bytes per bit target of a batch); larger inserts are processed in
 * batches, each of which reads and writes the index regions it touches.  The scratch is sized for
 * the first partitioned insert, kept by the handle, and released by the
 * next call of this function that changes scratch_bytes. */
#define RAMBO_INSERT_AUTO 0
#define RAMBO_INSERT_DIRECT 1
#define RAMBO_INSERT_PARTITIONED 2
/* PARTITIONED, with sequence input binned by the window-walker kernel (a
 * wave walks 64 consecutive bytes per step, whatever the sequence) instead
 * of the piece kernel (a wave walks pieces of one sequence, a lane a run of
 * windows); the same index bits, for comparing the two. */
#define RAMBO_INSERT_PARTITIONED_WALKER 3
int rambo_set_insert_policy(rambo_t *h, int mode, uint64_t scratch_bytes);

/* Tile shapes of the partitioned insert (the index bits are the same for
 * every choice; an autotuner picks them).  0 leaves a field automatic.
 *   steps:        windows each lane hashes per round of the piece stage A,
 *                 1 or 2 (automatic: 2 for R <= 5, 1 for R = 6; more steps
 *                 give longer runs per coarse bucket but need more registers)
 *   stage_b_tile: slab entries per stage-B tile, 8192, 16384 or 32768
 *                 (automatic: 32768 from 2048 regions per coarse bucket,
 *                 16384 from 1024, else 8192)
 *   groups:       groups of coarse buckets that stages B and C run over,
 *                 1, 2, 4 or 8 (automatic: the fewest that need the fewest
 *                 scratch batches; slab B holds one group's regions)
 *   fine_bits:    log2 of the 2^20-bit regions per coarse bucket, 8 to 12
 *                 (automatic: up to 11 while 256 coarse buckets remain, more
 *                 while a stage-A round gives a bucket fewer than 32
 *                 entries); must leave at most
 *                 4096 coarse buckets, else RAMBO_EINVAL
 * Values outside these sets give RAMBO_EINVAL; a stage-B tile whose LDS
 * does not fit the regions of a coarse bucket, and more groups than coarse
 * buckets, fall back to what fits (rambo_get_insert_tiles shows what is
 * used).  A change releases the insert scratch (as rambo_set_insert_policy
 * does), and applies from the next insert. */
typedef struct rambo_insert_tiles {
    uint32_t steps;
    uint32_t stage_b_tile;
    uint32_t groups;
    uint32_t fine_bits;
} rambo_insert_tiles;
int rambo_set_insert_tiles(rambo_t *h, const rambo_insert_tiles *tiles);

/* The shapes the partitioned insert uses now (after its last scratch
 * sizing): every field filled in. */
int rambo_get_insert_tiles(rambo_t *h, rambo_insert_tiles *out);

/* How rambo_query_seqs and rambo_query_seqs_ids schedule a batch of reads
 * (the answers are the same either way): WAVE_PER_READ runs one wavefront
 * per read; QUEUE splits the reads into work items of chunk_bytes bytes that
 * a persistent
 * grid of waves_per_cu wavefronts per compute unit takes from a work counter;
 * the chunks of one read AND their group masks into per-read state and the
 * last one expands the answer, so long and short reads share the GPU evenly
 * and a read stops probing once one chunk found a repetition empty.
 * chunk_bytes 0 = 512, waves_per_cu 0 = 16.  AUTO takes one wavefront per
 * read when the reads average at most 2 048 bytes, else the queue.  Both
 * keep per-read state (ID-list form, queue) in device memory owned by the
 * handle, grown on demand. */
#define RAMBO_QUERY_AUTO 0
#define RAMBO_QUERY_WAVE_PER_READ 1
#define RAMBO_QUERY_QUEUE 2
int rambo_set_query_policy(rambo_t *h, int mode, uint32_t chunk_bytes, uint32_t waves_per_cu);

/* Kernel timing.  While enabled, every kernel the handle launches is
 * bracketed by a pair of HIP events recorded on the caller's stream (do not
 * enable it under graph capture).  rambo_get_stage_times synchronises those
 * events and reports, for the kernels launched since the last call to it,
 * the total milliseconds per kernel name: names receives up to max_stages
 * NUL-terminated names of at most 47 characters in 48-byte slots, ms their
 * times and calls (host memory, nullable) the number of launches behind
 * each total; the return value is the number of distinct kernels (or a
 * negative error). */
int rambo_set_timing(rambo_t *h, int enable);
int rambo_get_stage_times(rambo_t *h, char *names, float *ms, uint32_t *calls, int max_stages);

/* Folding over (Sec. 5.2 and the appendix's parallel-indexing experiment):
 * B -> B/2 by OR-ing the filter of cell b + B/2 into the filter of cell b
 * in every repetition; the sets of cell b + B/2 then belong to cell b
 * (phi_r becomes phi_r mod B/2), the answers keep every true holder and the
 * index takes half the memory (row stride max(8, next_pow2(B/2)) bits).
 * Later inserts and queries use the folded partition.  B must be even and
 * no query server may be attached (RAMBO_EINVAL otherwise); RAMBO_ENOMEM
 * when the new index cannot be allocated (the old one is then kept).  Synchronous: waits for the work on `stream`,
 * then replaces the index; the handle's scratch and per-read state are
 * released (rambo_get_info reports the new layout).  Graphs captured from
 * this handle before the fold hold the old index and must be captured
 * again. */
int rambo_fold(rambo_t *h, hipStream_t stream);

/* Checkpoint: write the index to the file at path (created or replaced):
 * a header with the configuration and layout, the partition phi (R x K u16)
 * and the R x words_per_rep index words, all little-endian, through a
 * pinned host buffer.  Waits for the work on `stream` first.  The streaming
 * updates of Sec. 3.1 can resume from it.  RAMBO_EIO on a file error. */
int rambo_save(rambo_t *h, const char *path, hipStream_t stream);

/* Resume: create an index from a file rambo_save wrote (the same
 * configuration, hash multipliers from its seed, its partition and its
 * bits).  Synchronous.  RAMBO_EIO for a missing or short file, RAMBO_EINVAL
 * for a file that is not an index or does not match its configuration. */
int rambo_load(const char *path, rambo_t **out);

/* The configuration of the index (after folding, B is the folded one). */
int rambo_get_config(const rambo_t *h, rambo_config *out);

/* Zero every Bloom filter (an empty index with the same hashes).  Inserts,
 * queries and clears may be recorded into a HIP graph on `stream` (stream
 * capture) once each kind of call has run eagerly with its sizes, so that its
 * scratch exists; recorded inserts always read the regions they update back,
 * and recorded calls take no timing events. */
int rambo_clear(rambo_t *h, hipStream_t stream);

/* Layout of the index (see above). */
int rambo_get_info(const rambo_t *h, rambo_info *out);

/* Copy n_words words of the index, starting at word word_offset, to dst
 * (device or host memory; asynchronous on `stream` for device memory).
 * RAMBO_EINVAL if the range is outside the index. */
int rambo_copy_index(rambo_t *h, uint64_t word_offset, uint64_t n_words, void *dst, hipStream_t stream);

/* phi_r(i) for all r, i, copied to host memory out[r*K + i] (R*K entries).
 * Synchronous. */
int rambo_get_partition(rambo_t *h, uint32_t *out);

/* Number of set bits of every Bloom filter: out[r*B + b] (R*B uint64,
 * device memory) = ones of cell b of repetition r, the n_b of the filter's
 * fill (Sec. 2), as the false-positive expression of Lemma 4.1 uses it.
 * Asynchronous on `stream`. */
int rambo_fill_counts(rambo_t *h, uint64_t *out, hipStream_t stream);

/* Synchronise `stream`, then return and clear the sticky device error:
 * RAMBO_OK, RAMBO_ERANGE, RAMBO_ECODE or RAMBO_EOVERFLOW (in that order of
 * precedence when several were raised). */
int rambo_sync_status(rambo_t *h, hipStream_t stream);

/* Text of the last error of the handle (or of the last failed create when
 * h is NULL). */
const char *rambo_last_error(const rambo_t *h);

#ifdef __cplusplus
}
#endif

#endif /* RAMBO_H */
