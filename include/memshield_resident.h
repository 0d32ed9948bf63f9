/*
 * memshield_resident.h - the paper's own GPU design: a key that lives only in
 * the registers of a kernel that keeps running, fed through a ring in mapped
 * host memory.
 *
 * MemShield (section 4.4) creates its 256-bit key at start-up, places it in
 * the registers of a GPU kernel that is never terminated (ending it would
 * lose the key), and checks that the kernel never spills registers to GPU
 * local memory.  Host threads hand it pages through a circular buffer in
 * memory mapped between host and device (multiple producers, GPU workers as
 * consumers), and the pages themselves travel between system RAM and the
 * GPU.  This engine reproduces that design on the MI355X:
 *   - ms_resident_start launches one kernel that holds `workers` worker
 *     waves and one poller wave; the key goes through a 32-byte device
 *     buffer which the kernel zeroes as soon as every worker holds the key in
 *     scalar registers; the host copy is wiped as soon as it is on the GPU;
 *   - ms_resident_submit writes 64-byte descriptors (up to desc_pages pages
 *     each) into a ring in pinned host memory; any number of host threads may
 *     submit; each worker serves its own fixed share of the ring positions;
 *   - pages are in pinned, coherent host memory (ms_host_alloc of
 *     memshield_host.h, or hipHostMalloc with hipHostMallocCoherent), which
 *     is the paper's data path, or in device memory of the context's GPU
 *     (a page request then never waits for a kernel launch); the kernel
 *     reads and writes them while it runs; nonces follow the linear rule
 *     (virtual address, PID) of ms_nonce, which is the paper's, or come from
 *     an array of 12-byte nonces in device or pinned host memory;
 *   - an engine holds one key (the paper's design: it stays in every
 *     worker's registers) or, started with ms_resident_start_keys, up to
 *     MS_RESIDENT_MAX_KEYS keys taken from the context's key table (one per
 *     client, say), which each workgroup of the kernel keeps in its LDS; a
 *     descriptor names its key by index.  Either way the keys are wiped from
 *     device memory once every worker holds them and live on chip only;
 *   - completion is a word per ring slot written by the kernel into host
 *     memory and read by ms_resident_poll, with no GPU call on the way.
 * The cipher is the same as ms_encrypt_pages with the same key: output bytes
 * are identical.
 *
 * Bounded lifetime.  The kernel ends when ms_resident_stop asks it to, or by
 * itself after idle_limit_ms without a submission or a poll (0 = no limit).
 * After that the key is gone, ms_resident_alive reads 0 and submissions
 * return MS_ECLOSED; start a new engine.  The kernel is dispatched on an HSA
 * queue of its own, outside the HIP runtime: no HIP stream, and no
 * device-wide synchronization, waits for it, and other work on the device
 * proceeds beside it.  ms_shutdown stops the context's engines that are
 * still running; their handles are then invalid.
 */
#ifndef MEMSHIELD_RESIDENT_H
#define MEMSHIELD_RESIDENT_H

#include "memshield.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ms_resident ms_resident;  /* opaque */

#define MS_RESIDENT_MAX_KEYS 64

typedef struct ms_resident_config {
    uint32_t workers;        /* worker waves (default 256; at most 4 per
                                compute unit, minus one for the poller) */
    uint32_t ring_depth;     /* descriptors in the ring: power of two,
                                16..1048576 (default 4096) */
    uint32_t desc_pages;     /* pages per descriptor, 1..1024 (default 16) */
    uint32_t idle_limit_ms;  /* self-stop after this long idle (default
                                10000; 0 = never) */
    uint32_t reserved[4];
} ms_resident_config;

/* Fill `cfg` with the defaults above. */
void ms_resident_config_default(ms_resident_config *cfg);

/*
 * Start a resident-key engine on ctx's device with ctx's cipher and round
 * count (ms_config.cipher, .rounds).  `key` is 32 bytes, or NULL to draw
 * them with getrandom(2) straight into the library's pinned staging buffer
 * (the key is then known to no one).  Waits until every worker holds the
 * key and its memory copies are wiped.  Errors: MS_EINVAL, MS_ENOMEM,
 * MS_EDEVICE, MS_ETIMEDOUT (the kernel did not report ready within 10 s; it
 * is stopped).
 */
ms_status ms_resident_start(ms_ctx *ctx, const ms_resident_config *cfg,
                            const uint8_t *key, ms_resident **out);

/*
 * Start an engine that holds n_keys (1..MS_RESIDENT_MAX_KEYS) keys of the
 * context's key table: keys[i] becomes key index i of ms_resident_submit_keyed.
 * The key bytes are copied device to device (never through host memory);
 * the handles stay valid and usable on the context, and destroying one later
 * does not reach the engine's copy.  Errors as ms_resident_start, plus
 * MS_ENOKEY for an unknown handle.
 */
ms_status ms_resident_start_keys(ms_ctx *ctx, const ms_resident_config *cfg,
                                 const ms_key *keys, uint32_t n_keys,
                                 ms_resident **out);

/*
 * Queue n_pages pages from src to dst with key index 0;
 * ms_resident_submit_keyed with key_index 0.
 */
ms_status ms_resident_submit(ms_resident *r, const void *src, void *dst,
                             uint64_t n_pages, const ms_nonce *nonce,
                             ms_ticket *ticket_out);

/*
 * Queue n_pages pages from src to dst with the engine's key `key_index` and
 * a linear nonce, or an array of n_pages 12-byte nonces (device memory of
 * the context's GPU or pinned host memory, 4-byte aligned; it must stay
 * unchanged until the ticket is done).  src and dst are each pinned host memory or device memory
 * of the context's GPU, 16-byte aligned, src == dst or not overlapping.  The
 * request becomes ceil(n_pages / desc_pages) descriptors, queued together or
 * not at all; the ticket covers all of them.  Never blocks.  The kernel
 * does not wait for any stream: the source bytes must be complete when this
 * is called (synchronize the stream that produced them), and nothing may
 * read or write the destination until ms_resident_poll reports the ticket
 * done; from then on the pages are visible to the host and to later device
 * work.  Errors:
 * MS_EINVAL (a key index the engine does not hold, pageable or managed
 * memory, another GPU's memory, or more descriptors than the ring holds),
 * MS_EAGAIN (ring full now), MS_ECLOSED (the
 * kernel has stopped), MS_EDEVICE (the kernel rejected a descriptor).
 * Thread-safe.
 */
ms_status ms_resident_submit_keyed(ms_resident *r, uint32_t key_index,
                                   const void *src, void *dst,
                                   uint64_t n_pages, const ms_nonce *nonce,
                                   ms_ticket *ticket_out);

/*
 * done_out[i] = 1 when ticket i's pages are written, 0 while pending, or
 * MS_ECANCELED if the kernel stopped first.  Waits until all are done or
 * timeout_ns elapses (0 = just look), spinning on host memory.  Returns
 * MS_OK when none is pending, MS_ETIMEDOUT otherwise, MS_EINVAL for a
 * ticket this engine did not issue.  Thread-safe.
 */
ms_status ms_resident_poll(ms_resident *r, const ms_ticket *tickets, size_t n,
                           int32_t *done_out, uint64_t timeout_ns);

/* 1 while the kernel runs and holds the key, 0 after it stopped. */
int ms_resident_alive(ms_resident *r);

/*
 * Stop the kernel (the key is lost), wait for it to end, and free the
 * engine.  Requests still queued are not run.  NULL is a no-op.  Returns
 * MS_ETIMEDOUT if the kernel did not end within 60 s (the engine's buffers
 * are then left allocated).
 */
ms_status ms_resident_stop(ms_resident *r);

/*
 * Test hook for the key-purge property: 1 when both the device key buffer
 * (all the engine's keys) and the host staging buffer hold only zero bytes,
 * 0 otherwise, negative on error.
 */
int ms_resident_debug_key_wiped(ms_resident *r);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_RESIDENT_H */
