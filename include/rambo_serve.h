/*
 * rambo_serve.h - continuous-batching query server over a resident RAMBO
 * index (part of librambo.so).
 *
 * The index stays in device memory; requests (each a small batch of reads,
 * answered as in Sec. 3.2.1 of the RAMBO paper: the sets that hold every
 * k-mer of the read) are submitted from host memory at any time.  A worker
 * thread packs the queued requests into batches and runs them in "slots":
 * each slot owns a stream and mapped pinned staging (the device reads the
 * batch's reads from it and writes the K-bit answers and window counts
 * back into it: no copy-engine transfers); a batch's device buffers (read
 * bytes, offsets and the per-read state of the query kernels: 8 (n+2) +
 * bytes + 4 (n (R S/32 + 5) + 2) bytes for n reads, each part rounded up to
 * 256) come from one pool of mem_budget bytes, sized for what the batch
 * actually holds.  Admission is by free
 * device memory: a batch takes queued requests in order while the pool has
 * room for them, a request waits in the host queue while it has none, and
 * requests that arrive while other batches run are admitted as soon as
 * room and a slot free up, their batches overlapping on the GPU.  With
 * use_graphs each slot instead owns fixed buffers for the largest batch (a
 * replayed graph keeps its pointers), as many slots as mem_budget holds.
 * Each request's answer is the same whatever batch it shares (the per-read
 * computation does not depend on the other reads).
 *
 * While a server runs, its worker is the only thread that uses the index
 * handle; do not call other rambo_* functions on that handle until
 * rambo_serve_destroy returns.
 */
#ifndef RAMBO_SERVE_H
#define RAMBO_SERVE_H

#include <stdint.h>

#include "rambo.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RAMBO_ETIMEDOUT (-110)

typedef struct rambo_server rambo_server_t;

typedef struct rambo_serve_config {
    uint64_t mem_budget;       /* device bytes for the batches in flight (0 = 1 GiB) */
    uint64_t max_batch_bytes;  /* read bytes per batch (0 = 8 MiB) */
    uint32_t max_slots;        /* batches in flight at once, 1..16 (0 = 4) */
    uint32_t max_batch_reads;  /* reads per batch (0 = 8192) */
    uint32_t use_graphs;       /* replay one captured hipGraph per slot for the query kernels */
    uint32_t reserved;
} rambo_serve_config;

/* Start a server on index h (which must outlive it).  Allocates the pool
 * and max_slots slots (with use_graphs: as many slots as fit mem_budget, at
 * most max_slots) and starts the worker thread.  RAMBO_ENOMEM unless
 * mem_budget holds one batch of max_batch_reads reads and max_batch_bytes
 * bytes.  A batch takes queued requests while the pool has room, and past
 * its first request at most mem_budget / max_slots bytes, so that every
 * slot can run one. */
int rambo_serve_create(rambo_t *h, const rambo_serve_config *cfg, rambo_server_t **out);

/* Finish every queued and in-flight request, stop the worker, free the
 * slots.  NULL is a no-op. */
void rambo_serve_destroy(rambo_server_t *s);

/* Queue a request of n_reads reads given in HOST memory (offsets: n_reads+1
 * entries, non-decreasing, bytes chars[offsets[0] .. offsets[n_reads])).
 * The data are copied before the call returns.  Returns the request id
 * (>= 0), or RAMBO_EINVAL if the request is larger than one batch or than
 * the whole pool. */
int64_t rambo_serve_submit(rambo_server_t *s, const uint64_t *offsets, uint64_t n_reads, const uint8_t *chars);

/* Queue an insertion (Alg. 1; streaming updates, Sec. 3.1) of n_seqs
 * sequences given in HOST memory: every valid k-window of bytes
 * chars[offsets[s] .. offsets[s+1]) goes into set set_ids[s] (offsets:
 * n_seqs+1 entries, non-decreasing).  The data are copied before the call
 * returns.  Requests take effect in submission order: the insert waits for
 * every batch admitted before it and later requests wait for the insert, so
 * a query submitted before it is answered without its terms and one
 * submitted after it with them.  The insert uses atomic ORs into the index
 * and a device staging buffer of the server (grown to the largest insert).
 * Returns the request id (>= 0) or RAMBO_EINVAL; rambo_serve_wait on the id
 * returns the insert's status (RAMBO_ERANGE for a set id >= K: that
 * sequence is skipped). */
int64_t rambo_serve_submit_insert(rambo_server_t *s, const uint32_t *set_ids, const uint64_t *offsets,
                                  uint64_t n_seqs, const uint8_t *chars);

/* Wait up to timeout_us microseconds (-1: no limit) for request id; on
 * success copy its masks (n_reads x W words) and, if nkmers is not NULL, its
 * valid-window counts to host memory, store the time from submission to the
 * results reaching host memory in *latency_ms (if not NULL), and forget the
 * request.  RAMBO_ETIMEDOUT leaves it pending; RAMBO_EINVAL for an unknown
 * id.  For an insert request nothing is copied (masks and nkmers may be
 * NULL) and the insert's own status is returned. */
int rambo_serve_wait(rambo_server_t *s, int64_t id, uint32_t *masks, uint32_t *nkmers, double *latency_ms,
                     int64_t timeout_us);

/* Open-loop load driver (measurement): request i - the reads
 * req_reads[i] .. req_reads[i+1]-1 of the host CSR read_offsets / chars,
 * 1 to max_batch_reads reads - is submitted from a native thread at
 * arrival_s[i] seconds after the start (non-decreasing), while the calling
 * thread waits for the answers in order.  latency_ms[i] = arrival to answer
 * in host memory (the submit lag included); queue_ms[i] (if not NULL) =
 * arrival to the enqueue of its batch's work, the part of the latency spent
 * waiting on the host.  *checksum (if not NULL) hashes every answer word in
 * request order.  Returns RAMBO_OK or the first error; the requests already
 * submitted are answered either way. */
int rambo_serve_replay(rambo_server_t *s, uint64_t n_req, const uint64_t *req_reads, const uint64_t *read_offsets,
                       const uint8_t *chars, const double *arrival_s, double *latency_ms, double *queue_ms,
                       uint64_t *checksum);

/* Test hook of the worker's error path: the next n_batches batches fail on
 * the host before they are launched, exactly as a failed copy or launch
 * would: every request in them is answered with RAMBO_EHIP (zero masks)
 * instead of leaving its waiter blocked, and the server goes on with later
 * batches.  A batch whose completion event reports an error is handled the
 * same way. */
int rambo_serve_inject_failures(rambo_server_t *s, uint32_t n_batches);

/* Counters since creation: batches run, requests and reads answered, and the
 * number of slots. */
int rambo_serve_stats(rambo_server_t *s, uint64_t *batches, uint64_t *requests, uint64_t *reads, uint32_t *slots);

/* Timing of the worker thread (microseconds, maxima since creation or the
 * last reset): the longest time between two passes of its loop (time
 * spent blocked on an empty queue excluded), the longest enqueue of one
 * batch (copies and launches) and the longest completion query.  With
 * reset != 0 the maxima restart from zero after being read. */
int rambo_serve_worker_stats(rambo_server_t *s, double *max_loop_gap_us, double *max_enqueue_us,
                             double *max_query_us, int reset);

/* Device bytes of one batch of n_reads reads and n_bytes read bytes on index
 * h (for sizing mem_budget); 0 for a NULL handle. */
uint64_t rambo_serve_batch_bytes(const rambo_t *h, uint64_t n_reads, uint64_t n_bytes);

/* Device memory of the batches: the pool size, the bytes its batches hold
 * now and at most so far, and how many times a queued query waited for room
 * (with use_graphs: the slots' fixed buffers, and no waits). */
int rambo_serve_mem_stats(rambo_server_t *s, uint64_t *budget, uint64_t *in_use, uint64_t *peak, uint64_t *waits);

#ifdef __cplusplus
}
#endif

#endif /* RAMBO_SERVE_H */
