/*
 * rambo_roofline.h - probes of the memory system for the RAMBO access
 * patterns, part of librambo.so.
 *
 * The index is bound by scattered memory traffic, not arithmetic: a term
 * query reads R*eta rows at random positions (Alg. 2), an insertion ORs
 * R*eta bits at random positions (Alg. 1).  These probes measure what the
 * GPU sustains for exactly those patterns over a buffer as large as the
 * index, so that kernel throughput can be stated as a fraction of a measured
 * random-access ceiling next to the datasheet one.
 *
 * All pointers are device pointers owned by the caller; calls are
 * asynchronous on `stream` (host out-parameters are written before the
 * call returns); return 0 or RAMBO_EINVAL (rambo.h codes).
 */
#ifndef RAMBO_ROOFLINE_H
#define RAMBO_ROOFLINE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* n_access aligned reads of access_bytes (4, 8, 16, 32, 64, 128 or 256)
 * at uniformly random offsets of buf (buf_bytes long, a multiple of
 * access_bytes).  Offsets come from mix64(seed + i).  The loaded data are
 * folded into one word that is written to *sink only if it equals an
 * improbable constant, so no load can be dropped. */
int rambo_roofline_gather(const void *buf, uint64_t buf_bytes, uint32_t access_bytes, uint64_t n_access,
                          uint64_t seed, uint32_t *sink, hipStream_t stream);

/* n_access non-returning 32-bit atomicOr of one random bit at uniformly
 * random words of buf (buf_words words). */
int rambo_roofline_atomic_or(uint32_t *buf, uint64_t buf_words, uint64_t n_access, uint64_t seed,
                             hipStream_t stream);

/* The write pattern of the partitioned insert's binning (stage A): each of
 * n_workgroups workgroups of 1024 threads owns a chunk of every one of
 * `streams` buckets of buf (buf_words words; chunk (b, g) holds cap =
 * buf_words / (streams * n_workgroups) words, rounded down to a multiple of
 * 16) and each round appends a run of `run` 32-bit words to each of its
 * chunks, consecutive lanes writing consecutive words, for as many rounds as
 * fit.  With `misaligned` != 0 every chunk's runs start 0..15 words into its
 * first 64-byte segment (from mix64 of the bucket and the workgroup), so runs
 * start and end inside segments as appends at a running cursor do; with 0
 * every run of 16 words fills one aligned segment.  *written_words (host
 * memory) receives the words the launch writes.  RAMBO_EINVAL for a null
 * pointer, a zero count, streams * run above 2^32 - 1 or a chunk that cannot
 * hold one run. */
int rambo_roofline_append(uint32_t *buf, uint64_t buf_words, uint32_t streams, uint32_t run, uint32_t misaligned,
                          uint32_t n_workgroups, uint64_t *written_words, hipStream_t stream);

/* Streaming copy of bytes (a multiple of 16) from src to dst: the
 * sequential-bandwidth reference and the calibration kernel of the memory
 * counters (it reads and writes exactly `bytes` each). */
int rambo_roofline_copy(const void *src, void *dst, uint64_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RAMBO_ROOFLINE_H */
