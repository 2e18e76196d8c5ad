/*
 * rambo_serve.h - continuous-batching query server over a resident RAMBO
 * index (part of librambo.so).
 *
 * The index stays in device memory; requests (each a small batch of reads,
 * answered as in Sec. 3.2.1 of the RAMBO paper: the sets that hold every
 * k-mer of the read) are submitted from host memory at any time.  A worker
 * thread packs the queued requests into batches and runs them in "slots":
 * each slot owns a stream, pinned staging, device buffers for read bytes,
 * offsets, K-bit result masks and the per-read state of the work-queue
 * kernel.  The slots are carved from a device-memory budget, so admission is
 * by free device memory: a request waits in the host queue until a slot is
 * free, and requests that arrive while other batches run are admitted as soon
 * as a slot frees up, their batches overlapping on the GPU.  Each request's
 * answer is the same whatever batch it shares (the per-read computation does
 * not depend on the other reads).
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
    uint64_t mem_budget;       /* device bytes for all slots (0 = 1 GiB) */
    uint64_t max_batch_bytes;  /* read bytes per batch (0 = 8 MiB) */
    uint32_t max_slots;        /* batches in flight at once, 1..16 (0 = 4) */
    uint32_t max_batch_reads;  /* reads per batch (0 = 8192) */
    uint32_t use_graphs;       /* replay one captured hipGraph per slot for the query kernels */
    uint32_t reserved;
} rambo_serve_config;

/* Start a server on index h (which must outlive it).  Allocates the slots
 * (as many as fit mem_budget, at most max_slots; at least one, else
 * RAMBO_ENOMEM) and starts the worker thread. */
int rambo_serve_create(rambo_t *h, const rambo_serve_config *cfg, rambo_server_t **out);

/* Finish every queued and in-flight request, stop the worker, free the
 * slots.  NULL is a no-op. */
void rambo_serve_destroy(rambo_server_t *s);

/* Queue a request of n_reads reads given in HOST memory (offsets: n_reads+1
 * entries, non-decreasing, bytes chars[offsets[0] .. offsets[n_reads])).
 * The data are copied before the call returns.  Returns the request id
 * (>= 0), or RAMBO_EINVAL if the request is larger than one batch. */
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
 * in host memory (the submit lag included).  *checksum (if not NULL) hashes
 * every answer word in request order.  Returns RAMBO_OK or the first error;
 * the requests already submitted are answered either way. */
int rambo_serve_replay(rambo_server_t *s, uint64_t n_req, const uint64_t *req_reads, const uint64_t *read_offsets,
                       const uint8_t *chars, const double *arrival_s, double *latency_ms, uint64_t *checksum);

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

#ifdef __cplusplus
}
#endif

#endif /* RAMBO_SERVE_H */
