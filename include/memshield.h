/*
 * memshield.h - C ABI of the MI355X page-cipher engine.
 *
 * The engine implements the GPU half of MemShield (Santucci et al., "GPU-
 * assisted software memory encryption", ACNS 2020): bulk encryption and
 * decryption of 4096-byte memory pages with ChaCha20, the key living only in
 * GPU memory.  The paper's problem statement (section 4.4): every
 * cryptographic operation works on one page of 4096 bytes; the page is XORed
 * with 64-byte ChaCha20 keystream blocks; the 384-bit seed of each block is a
 * 256-bit key created once from the operating system's CSPRNG, sent to the
 * GPU and purged from host memory, plus a 128-bit value made of the page's
 * virtual address, the client's PID and a counter 0..63 that is the block's
 * index in the page; encryption and decryption are the same operation; many
 * host threads submit pages concurrently (multiple producers, one consumer
 * per GPU worker).
 *
 * Layout of one keystream block (ChaCha as published by Bernstein, 2008, in
 * the 96-bit-nonce form): state word 12 is the block counter j = 0..63, words
 * 13..15 are the page's 12-byte nonce read as three little-endian words.
 * Ciphertext byte 64*j+i of a page is plaintext byte 64*j+i XOR keystream
 * byte i of block j.
 *
 * Conventions for every call:
 *   - status codes are returned, never thrown; out-parameters are written only
 *     when the call returns MS_OK;
 *   - page buffers (src, dst) and nonce arrays are DEVICE memory owned by the
 *     caller (e.g. a torch tensor's data_ptr()); they must stay valid until
 *     the work that reads them has completed (stream order for the
 *     synchronous-issue calls, ms_poll for submitted requests);
 *   - page buffers must be 16-byte aligned, nonce arrays 4-byte aligned;
 *     src == dst (in place) is allowed, any other overlap is MS_EINVAL;
 *   - with pointer validation on (the default) every device range is checked
 *     against the allocation that holds it, so a size that runs past the end
 *     of the caller's allocation is MS_EINVAL instead of a GPU fault;
 *   - a `stream` argument is a hipStream_t passed as void*; NULL selects the
 *     context's own stream;
 *   - an error raised by the GPU is reported as MS_EDEVICE by the next call
 *     that notices it;
 *   - key bytes are never returned by any call.
 */
#ifndef MEMSHIELD_H
#define MEMSHIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MS_ABI_VERSION 1
#define MS_PAGE_SIZE 4096u       /* section 4.4: one page per operation */
#define MS_BLOCK_SIZE 64u        /* 512-bit keystream block */
#define MS_BLOCKS_PER_PAGE 64u   /* block counter range 0..63 */
#define MS_KEY_BYTES 32u         /* 256-bit key */
#define MS_NONCE_BYTES 12u       /* 96-bit page nonce (seed words 13..15) */

typedef struct ms_ctx ms_ctx;    /* opaque engine context, one per GPU */
typedef uint64_t ms_key;         /* opaque key handle; 0 is never valid */
typedef uint64_t ms_ticket;      /* opaque request ticket; 0 is never valid */

typedef enum ms_status {
    MS_OK = 0,
    MS_EINVAL = -1,      /* bad argument, size, alignment, overlap or range */
    MS_ENOKEY = -2,      /* unknown, destroyed or stale key handle */
    MS_ENOMEM = -3,      /* allocation failed, or key table full */
    MS_EAGAIN = -4,      /* queue full or admission cap reached; retry */
    MS_EBUSY = -5,       /* key still referenced by requests in flight */
    MS_EDEVICE = -6,     /* the GPU or the HIP runtime reported an error */
    MS_ECLOSED = -7,     /* context is shutting down */
    MS_ETIMEDOUT = -8,   /* ms_poll timed out with requests pending */
    MS_ENOTSUP = -9,     /* option not supported by this entry point */
    MS_ECANCELED = -10   /* request cancelled (client cancelled or dropped) */
} ms_status;

typedef enum ms_op { MS_ENCRYPT = 0, MS_DECRYPT = 1 } ms_op;

/*
 * Page nonces.  MS_NONCE_ARRAY: `array` is a device buffer of n_pages*12
 * bytes, page p using bytes 12p..12p+11.  MS_NONCE_LINEAR: page p of the run
 * uses LE64(base + p*stride mod 2^64) || LE32(tag); with base = the virtual
 * address of the run's first page, stride = 4096 and tag = the client's PID
 * this is the paper's seed value (virtual address, PID; the counter is
 * internal).
 */
typedef enum ms_nonce_kind { MS_NONCE_ARRAY = 0, MS_NONCE_LINEAR = 1 } ms_nonce_kind;

typedef struct ms_nonce {
    int32_t kind;            /* ms_nonce_kind */
    uint32_t tag;            /* LINEAR: word 15 of the state */
    const uint8_t *array;    /* ARRAY: device pointer, 4-byte aligned */
    uint64_t base;           /* LINEAR: nonce of page 0 (words 13..14) */
    uint64_t stride;         /* LINEAR: increment per page */
} ms_nonce;

/* One encrypt/decrypt job over a run of consecutive pages. */
typedef struct ms_request {
    int32_t op;              /* ms_op; informational, both run the same XOR */
    uint32_t client;         /* caller's client id (for cancellation, stats) */
    ms_key key;
    const void *src;         /* device, n_pages*4096 bytes, 16-B aligned */
    void *dst;               /* device, same size; == src for in place */
    uint64_t n_pages;        /* >= 1 for submitted requests */
    ms_nonce nonce;
    uint32_t priority;       /* reserved, must be 0 */
    uint32_t flags;          /* reserved, must be 0 */
} ms_request;

typedef struct ms_config {
    uint32_t max_keys;            /* key-table slots (default 64, max 65536) */
    uint32_t rounds;              /* cipher rounds: 20 (default), 12 or 8 */
    uint32_t queue_depth;         /* max submitted, not yet completed requests
                                     (default 65536, power of two) */
    uint32_t max_batch_requests;  /* requests per fused launch (default 1024) */
    uint64_t admission_cap_bytes; /* page bytes in flight on the device
                                     (default 8 GiB) */
    uint32_t inflight_batches;    /* batches on the device at once (default 4) */
    uint32_t prefetch_depth;      /* queued prefetch hints (default 4096) */
    uint32_t validate_pointers;   /* 1 (default): check every device range */
    uint32_t use_graphs;          /* 1 (default): ms_process_batch replays a
                                     captured hipGraph of its descriptor copy
                                     and batch kernel; 0: it launches
                                     directly, a batch of at most 15
                                     requests as one kernel with its records
                                     in the arguments (the serving
                                     scheduler always launches directly) */
    uint32_t host_chunk_pages;    /* staged host-page calls: pages per chunk
                                     (default 16384, at most 65536) */
    uint32_t host_stage_slots;    /* staged host-page calls: device staging
                                     buffers of one chunk (default 3, 2..16) */
    uint32_t host_mapped_waves;   /* kernels that read or write host pages:
                                     at most this many waves, so that few
                                     reads wait on the link (default 128) */
    uint32_t serve_spin_us;       /* the scheduler polls this long after its
                                     last work before it sleeps until the
                                     next submission (default 5000) */
    uint32_t cipher;              /* MS_CIPHER_CHACHA (default, the paper's
                                     cipher) or MS_CIPHER_SALSA (Salsa20,
                                     see below); every page kernel of the
                                     context uses it */
    uint32_t serve_stage;         /* how ms_submit / ms_prefetch_hint run
                                     their requests: MS_SERVE_STAGE_AUTO
                                     (default), _LAUNCH or _RING, below */
} ms_config;

/*
 * Serving stages.  MS_SERVE_STAGE_LAUNCH: a scheduler thread forms fused
 * launches from the queued requests on the context's serving streams
 * (continuous batching by launches).  MS_SERVE_STAGE_RING: requests of at
 * most 1024 pages go to a resident kernel on an HSA queue of the context's
 * own (the paper's never-ending kernel fed through memory mapped between
 * host and device, section 4.4): the submitting thread writes one
 * descriptor per page into a ring in pinned memory, the kernel's workers,
 * one wave per position of their share, read each descriptor's key from
 * the context's device key table, cipher the page and write a completion
 * word that ms_poll reads directly; requests that arrive while others run
 * are served at once by idle workers.  Longer requests still go to fused
 * launches.  The kernel starts with the first submission (about one
 * workgroup of 4 waves on every compute unit) and runs until ms_shutdown.
 * Prefetch hints enter the ring only while no demand request waits and at
 * most half of the workers hold work.  The ring runs the context's cipher
 * and round count.  MS_SERVE_STAGE_AUTO: the ring.
 */
#define MS_SERVE_STAGE_AUTO 0u
#define MS_SERVE_STAGE_LAUNCH 1u
#define MS_SERVE_STAGE_RING 2u

/*
 * The context's stream cipher.  Sections 1 and 6 of the paper make the
 * cipher a replaceable module; ChaCha (section 4.4) is the default.
 * MS_CIPHER_SALSA is Salsa20 (Bernstein 2008) with `rounds` rounds over the
 * same page interface: for page nonce N (12 bytes) block j of the page is
 * the Salsa20 block with the 64-bit nonce N[0..7] and the 64-bit block
 * counter LE32(N[8..11]) * 2^32 + j.  Every path runs it: plain and
 * batched launches, host-page modes, both serving stages and the
 * resident-key engine (memshield_resident.h).
 */
#define MS_CIPHER_CHACHA 0u
#define MS_CIPHER_SALSA 1u

/* Tunables of the fused batched launch, chosen by ms_autotune. */
typedef struct ms_tuning {
    uint32_t pages_per_wave;      /* pages a wave takes per work item */
    uint32_t unroll;              /* pages a wave ciphers at once: 1 or 2 */
    uint32_t waves_per_cu;        /* grid size in waves per compute unit */
    uint32_t reserved;
    double us_per_launch;         /* measured time of the winning candidate */
} ms_tuning;

typedef struct ms_stats {
    uint64_t submitted;           /* requests accepted by ms_submit */
    uint64_t completed;           /* requests finished on the device */
    uint64_t rejected_eagain;     /* submissions refused with MS_EAGAIN */
    uint64_t batches;             /* fused launches issued on the launch
                                     stage (the ring stage forms none) */
    uint64_t pages;               /* pages of the requests served, either
                                     stage */
    uint64_t prefetch_issued;     /* prefetch hints executed */
    uint64_t prefetch_dropped;    /* prefetch hints dropped */
    uint64_t cancelled;           /* requests cancelled before launch */
    uint64_t inflight_bytes;      /* page bytes currently admitted */
    uint64_t max_inflight_bytes;  /* high-water mark of inflight_bytes */
    uint64_t max_batch_requests;  /* largest batch formed */
    uint64_t max_inflight_batches;/* most fused launches on the device at once */
    uint64_t ring_direct;         /* ring stage: requests published by their
                                     submitting thread at once */
    uint64_t ring_queued;         /* ring stage: requests that waited in the
                                     client queues */
    uint64_t ring_max_queued;     /* high-water mark of those queues */
    uint64_t ring_reap_ns;        /* time in ring reaping passes that
                                     finished at least one request */
} ms_stats;

/* Fill `cfg` with the defaults listed in ms_config. */
void ms_config_default(ms_config *cfg);

/* Text for a status code; never NULL, static storage. */
const char *ms_status_str(ms_status st);

/*
 * Create a context on HIP device `hip_device`: allocates the device key table
 * (max_keys x 32 bytes, zeroed), a pinned 32-byte key staging buffer, the
 * context stream and the batch/serving machinery, and starts the scheduler
 * thread.  `cfg` may be NULL for defaults.  Errors: MS_EINVAL (bad config or
 * device), MS_ENOMEM, MS_EDEVICE.
 */
ms_status ms_init(ms_ctx **out, int hip_device, const ms_config *cfg);

/*
 * Drain submitted work, zero the device key table, free everything.  Must
 * not run concurrently with any other call on the same context.  NULL is a
 * no-op.
 */
ms_status ms_shutdown(ms_ctx *ctx);

/*
 * Key lifecycle (section 4.4: key from the OS CSPRNG, sent to the GPU, purged
 * from host memory).  ms_key_load copies the caller's 32 bytes through the
 * library's pinned staging buffer into a free device key slot and wipes the
 * staging buffer before returning (the caller's buffer is the caller's to
 * wipe).  ms_key_generate draws the 32 bytes with getrandom(2) straight into
 * the staging buffer, so the key is never in any other host memory.
 * ms_key_destroy waits for device work, zeroes the slot and invalidates the
 * handle; it returns MS_EBUSY while submitted requests still use the key.
 * Errors: MS_EINVAL, MS_ENOMEM (table full), MS_ENOKEY, MS_EBUSY,
 * MS_EDEVICE.  Key calls are serialized internally.
 */
ms_status ms_key_load(ms_ctx *ctx, const uint8_t key[32], ms_key *out);
ms_status ms_key_generate(ms_ctx *ctx, ms_key *out);
ms_status ms_key_destroy(ms_ctx *ctx, ms_key key);

/*
 * Encrypt (decrypt) n_pages consecutive pages from `src` to `dst` with `key`
 * and `nonce`, as one plain launch enqueued on `stream`.  Returns once the
 * launch is enqueued.  n_pages == 0 is a no-op returning MS_OK.  The two
 * calls produce identical bytes (section 4.4: same operation both ways).
 * Errors: MS_EINVAL, MS_ENOKEY, MS_EDEVICE.
 */
ms_status ms_encrypt_pages(ms_ctx *ctx, ms_key key, const void *src, void *dst,
                           uint64_t n_pages, const ms_nonce *nonce,
                           void *stream);
ms_status ms_decrypt_pages(ms_ctx *ctx, ms_key key, const void *src, void *dst,
                           uint64_t n_pages, const ms_nonce *nonce,
                           void *stream);

/*
 * What ms_encrypt_pages / ms_decrypt_pages launch for a call of n_pages
 * pages with nonces of `nonce_kind` on this context: the kernel, named with
 * its template arguments as a profiler prints it (cipher, rounds, pages in
 * flight per wave, nonce kind), its grid and the number of launches.  For
 * reports and profiles; it launches nothing.  Errors: MS_EINVAL.
 */
typedef struct ms_launch_info {
    char kernel[96];          /* e.g. "plain_pages_kernel<0u, 20, 2, 1u>" */
    uint32_t launches;        /* launches of one call (at most 2^24 pages
                                 each) */
    uint32_t grid_blocks;     /* workgroups of the first launch */
    uint32_t block_threads;   /* threads per workgroup */
    uint32_t waves_per_cu;    /* resident waves per compute unit */
    uint32_t cipher, rounds, unroll, nonce_kind;
} ms_launch_info;

ms_status ms_plain_launch_info(ms_ctx *ctx, uint64_t n_pages,
                               int32_t nonce_kind, ms_launch_info *out);

/*
 * Run n requests, each with its own key, nonce and page count, as ONE fused
 * persistent launch enqueued on `stream`, using the tuning that ms_autotune
 * picked for a batch of this size (or the built-in default).  The request
 * descriptors go from a pinned host buffer of the context to device memory
 * through a small copy kernel on the same stream, ahead of the batch kernel;
 * with use_graphs on, the two are one replay of a captured hipGraph.  Requests with n_pages == 0 are
 * skipped.  Destinations must not overlap each other or any source other
 * than their own.  Returns once enqueued; the request array may be reused at
 * once.  At most max_batch_requests requests.  Errors: MS_EINVAL, MS_ENOKEY,
 * MS_EDEVICE.
 */
ms_status ms_process_batch(ms_ctx *ctx, const ms_request *reqs, size_t n,
                           void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fused
 * launch of ms_process_batch, with the same checks and the same bytes out,
 * that allocates nothing.  Its request descriptors (a 64-byte header plus 64
 * bytes per request) go to a device array of fixed size built into the
 * library, one per GPU, held until the process ends, through a pinned host
 * buffer that ms_init allocated; the kernel is launched directly (no graph)
 * on `stream` after the descriptor copy kernel on the same stream (a batch
 * of at most 15 requests is one kernel with its records in the kernel
 * arguments).  At most MS_STATIC_BATCH_MAX_REQUESTS requests (256 KiB of
 * descriptors), else MS_EINVAL.  Before it reuses the host buffer, a call
 * waits on the host until the previous call's copy and kernel are done.
 * Calls on one GPU share the device array: calls on different streams that
 * overlap on the device race (the later copy may overwrite descriptors that
 * the earlier kernel still reads), so order them on one stream or
 * synchronize between them; this holds across contexts on the same GPU.
 * Ownership of pages and nonce arrays as for ms_process_batch.
 * Errors: MS_EINVAL, MS_ENOKEY, MS_ENOTSUP, MS_EDEVICE.
 */
#define MS_STATIC_BATCH_MAX_REQUESTS 4096u
ms_status ms_process_batch_static(ms_ctx *ctx, const ms_request *reqs,
                                  size_t n, void *stream);

/*
 * Asynchronous serving path (continuous batching).  ms_submit validates the
 * requests and queues them; it never blocks.  The engine runs submitted work
 * on its own streams, which do not wait for the caller's streams: a
 * request's source bytes (and nonce array) must be complete, and no other
 * work may still be writing its destination, when ms_submit is called
 * (e.g. synchronize the stream that produced them first).  Admission keeps
 * the page bytes in flight within admission_cap_bytes on either serving
 * stage (ms_config.serve_stage):
 *   - ring stage: a request of at most 1024 pages is published by the
 *     submitting thread at once (one descriptor per page into the ring of a
 *     resident kernel) when nothing waits and the ring has free positions;
 *     otherwise it waits in its client's queue (ms_request.client), and the
 *     queues are published round robin, one request per client per turn,
 *     each client's requests in submission order;
 *   - launch stage (and requests above 1024 pages): a scheduler thread
 *     forms fused launches while a batch slot is free, so batches that
 *     arrive while others run overlap on the device.
 * tickets_out[i] receives a ticket per
 * request.  All-or-nothing: on any error no request of the call is queued.
 * Errors: MS_EINVAL, MS_ENOKEY, MS_EAGAIN (queue full), MS_ECLOSED.
 * Thread-safe: any number of threads may submit and poll at once.
 */
ms_status ms_submit(ms_ctx *ctx, const ms_request *reqs, size_t n,
                    ms_ticket *tickets_out);

/*
 * Completion of tickets.  done_out[i] = 1 when ticket i's pages are written,
 * 0 while pending, or a negative ms_status if it failed or was cancelled.
 * Waits until all are done or `timeout_ns` elapses (0 = just look).  Returns
 * MS_OK when none is pending, MS_ETIMEDOUT otherwise; MS_EINVAL for a ticket
 * that was never issued.  A ticket stays queryable until queue_depth newer
 * requests have completed; after that it reads as done.
 */
ms_status ms_poll(ms_ctx *ctx, const ms_ticket *tickets, size_t n,
                  int32_t *done_out, uint64_t timeout_ns);

/*
 * Low-priority, droppable decrypts (pre-decryption of pages a predictor
 * expects to be touched next).  Hints run only when no demand request is
 * waiting and the admission cap allows; a hint that finds the prefetch queue
 * full is dropped at once.  tickets_out may be NULL; a dropped hint's ticket
 * reads MS_ECANCELED.  Errors: MS_EINVAL, MS_ENOKEY, MS_ECLOSED.
 */
ms_status ms_prefetch_hint(ms_ctx *ctx, const ms_request *reqs, size_t n,
                           ms_ticket *tickets_out);

/*
 * Cancel every queued (not yet launched) request of `client`; their tickets
 * read MS_ECANCELED.  Requests already on the device complete normally.
 * `n_cancelled` may be NULL.
 */
ms_status ms_cancel_client(ms_ctx *ctx, uint32_t client, uint64_t *n_cancelled);

/* Block until every submitted request has completed (or failed). */
ms_status ms_drain(ms_ctx *ctx, uint64_t timeout_ns);

/*
 * Autotuner for the fused launch: times candidate (pages_per_wave, unroll,
 * waves_per_cu) tiles on a scratch batch of `n_pages` pages in device memory
 * the library allocates and frees, keeps the fastest for the size bucket of
 * n_pages (power-of-two buckets) and returns it in `out` (may be NULL).
 * Results are cached in memory and, when the environment variable
 * MS_TUNE_CACHE names a file, in that JSON file keyed by device name, compute
 * unit count and bucket.  Errors: MS_EINVAL, MS_ENOMEM, MS_EDEVICE.
 */
ms_status ms_autotune(ms_ctx *ctx, uint64_t n_pages, ms_tuning *out);

/* Current tuning for a batch of n_pages (tuned or default). */
ms_status ms_get_tuning(ms_ctx *ctx, uint64_t n_pages, ms_tuning *out);

/*
 * Force a tuning for every bucket (tests and sweeps); NULL restores tuning.
 * While a tuning is forced, the serving scheduler runs every batch with the
 * fused kernel and that tuning, also a batch of a single request (which it
 * otherwise runs with the plain kernel).
 */
ms_status ms_set_tuning(ms_ctx *ctx, const ms_tuning *t);

ms_status ms_get_stats(ms_ctx *ctx, ms_stats *out);

/*
 * Test hook for the key-purge property: 1 when the library's pinned key
 * staging buffer holds only zero bytes, 0 otherwise, negative on error.
 */
int ms_debug_staging_is_zero(ms_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_H */
