/*
 * memshield_serve.h - native load generator for the serving path.
 *
 * Replays a request trace (arrival times, sizes, clients, operations) against
 * one engine context and measures per-request latency the way a client sees
 * it: from the request's arrival time to the moment the client observes its
 * completion.  It exists in native code so that timing is not distorted by
 * the Python interpreter.  Two modes:
 *   MS_SERVE_BATCHED - client threads call ms_submit at each arrival; the
 *     context's serving stage runs them (continuous batching: fused
 *     launches formed by the scheduler, or the ring of a resident kernel,
 *     as ms_config.serve_stage says); a poller thread observes completion
 *     with ms_poll;
 *   MS_SERVE_PLAIN - one dispatcher thread issues each request at its arrival
 *     as its own plain launch (ms_encrypt_pages) on one stream, records an
 *     event after it, and a poller observes the events in order: the
 *     one-launch-per-request baseline;
 *   MS_SERVE_RESIDENT - no launch per request: the run starts a resident-key
 *     engine (memshield_resident.h) holding every client's key (copied from
 *     the context's key table; at most MS_RESIDENT_MAX_KEYS clients), with
 *     one descriptor per page and 4 * compute units - 1 workers; client
 *     threads submit each request into its ring at arrival, a poller
 *     observes completion words in host memory, and the engine is stopped
 *     at the end.  This is the paper's own serving design (a kernel that
 *     never ends, fed through a ring in mapped memory) on device pages.
 * Before the first arrival each mode runs one warm-up request (the first
 * page of request 0) through its own path and waits for it, so that
 * one-time costs (the serving stage's start, a first launch) stay out of
 * the measured latencies.
 * The paper's server handles many clients' page requests concurrently
 * through per-worker multiple-producer queues (section 4.4); this harness
 * drives the engine's equivalent with synthetic traffic.
 */
#ifndef MEMSHIELD_SERVE_H
#define MEMSHIELD_SERVE_H

#include "memshield.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ms_serve_mode {
    MS_SERVE_BATCHED = 0,
    MS_SERVE_PLAIN = 1,
    MS_SERVE_RESIDENT = 2
} ms_serve_mode;

/* Host arrays of n entries each (request i). */
typedef struct ms_serve_trace {
    uint64_t n;
    const double *arrival_s;   /* non-decreasing, seconds from start */
    const uint32_t *client;    /* index into the keys array */
    const int32_t *op;         /* ms_op */
    const uint64_t *n_pages;   /* >= 1 */
    const uint64_t *src_page;  /* first page of the input in src_pool */
    const uint64_t *dst_page;  /* first page of the output in dst_pool */
    const uint64_t *va;        /* nonce base (virtual address of page 0) */
    const uint32_t *pid;       /* nonce tag */
} ms_serve_trace;

typedef struct ms_serve_result {
    double wall_s;             /* first arrival to last observed completion */
    double data_gbps;          /* page bytes processed / wall_s / 1e9 */
    double mean_us, p50_us, p90_us, p99_us, p999_us, max_us;
    double late_submit_us_max; /* worst lateness of a submission */
    uint64_t completed;
    uint64_t eagain_retries;   /* MS_EAGAIN answers that were retried */
    uint64_t failed;           /* requests that completed with an error */
    uint64_t first_failed;     /* 1 + index of the first failed request,
                                  0 if none */
    int64_t first_failed_state;/* its completion state (an ms_status) */
    double submit_call_p50_us; /* time inside the submitting call (ms_submit,
                                  the resident submit, or the launch and its
                                  event record), median and 99th percentile */
    double submit_call_p99_us;
} ms_serve_result;

/*
 * Run the trace.  src_pool / dst_pool are device buffers of
 * src_pool_pages / dst_pool_pages pages; every request must fit inside them
 * (MS_EINVAL otherwise, checked before anything runs).  keys[client] is the
 * key of each client.  submit_threads client threads share the arrivals in
 * batched and resident modes (1..64).  latency_us_out (may be NULL) receives n latencies,
 * arrival to observed completion.  Pages a request writes must not be read
 * or written by any request still in flight (the caller lays out dst).
 * Errors: MS_EINVAL, MS_EDEVICE, MS_ETIMEDOUT (a request did not complete
 * within 60 s of the last arrival).
 */
ms_status ms_serve_run(ms_ctx *ctx, const ms_serve_trace *trace,
                       const ms_key *keys, uint32_t n_keys,
                       const void *src_pool, uint64_t src_pool_pages,
                       void *dst_pool, uint64_t dst_pool_pages,
                       int32_t mode, uint32_t submit_threads,
                       double *latency_us_out, ms_serve_result *result);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_SERVE_H */
