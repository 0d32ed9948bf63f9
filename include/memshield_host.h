/*
 * memshield_host.h - pages that live in host memory.
 *
 * In MemShield both ends of every cryptographic operation sit in system RAM
 * (sections 4.2 and 4.3): the server keeps the encrypted copies of a client's
 * pages in its own address space, hands a decrypted page back to the faulting
 * client, and receives the clear contents of a page leaving the sliding
 * window for encryption.  Each such page crosses the host-GPU link twice, a
 * cost the evaluation (section 6) calls intrinsic to the design.  These calls
 * run the same page cipher as ms_encrypt_pages, with either buffer in pinned
 * host memory; the link (PCIe), not the GPU, bounds them.
 *
 * Host buffers must be pinned and mapped into the GPU's address space: memory
 * from ms_host_alloc, hipHostMalloc, or a torch tensor created with
 * pin_memory=True.  Pageable memory (malloc, numpy) is rejected with
 * MS_EINVAL: pin it by copying it into such a buffer.  Nonce arrays stay in
 * device memory, as for every other call.
 *
 * Three ways to move the bytes, chosen per call:
 *   MS_HOST_MAPPED  the cipher kernel reads and writes the host pages
 *                   directly through the link (zero copy).  One launch, no
 *                   staging; reads and writes share the link in both
 *                   directions at once.
 *   MS_HOST_DMA     the copy engines move chunks of pages host->device into
 *                   library-owned device staging buffers, the kernel ciphers
 *                   them there, and the copy engines move them back; the
 *                   three steps of successive chunks overlap on three
 *                   streams.
 *   MS_HOST_DMA_IN  copy engines inbound, the kernel writes the host
 *                   destination directly.
 * MS_HOST_AUTO selects MS_HOST_MAPPED: with its wave count capped
 * (ms_config.host_mapped_waves) it matches or passes the staged pipeline at
 * every run size on an MI355X host link, and has the lowest latency.
 * Whatever the mode, the output bytes are identical to those of
 * ms_encrypt_pages on the same key, nonce and input.
 */
#ifndef MEMSHIELD_HOST_H
#define MEMSHIELD_HOST_H

#include "memshield.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ms_host_mode {
    MS_HOST_AUTO = 0,
    MS_HOST_MAPPED = 1,
    MS_HOST_DMA = 2,
    MS_HOST_DMA_IN = 3
} ms_host_mode;

/*
 * Allocate `bytes` (> 0) of pinned, GPU-mapped, coherent (fine-grained) host
 * memory, zero-filled, for use as page buffers of the calls below and of
 * the resident-key engine.  *out receives the address (valid
 * on the host and, through the same address, on the GPU).  Errors:
 * MS_EINVAL, MS_ENOMEM.
 */
ms_status ms_host_alloc(ms_ctx *ctx, uint64_t bytes, void **out);

/*
 * Overwrite a buffer from ms_host_alloc with zeros (clear pages must not
 * outlive their use in RAM, section 4.3) and release it.  The caller must not
 * free a buffer that enqueued work still uses.  Errors: MS_EINVAL for a
 * pointer that ms_host_alloc of this context did not return.
 */
ms_status ms_host_free(ms_ctx *ctx, void *p);

/*
 * Encrypt (decrypt) n_pages consecutive 4096-byte pages from `src` to `dst`
 * with `key` and `nonce`, where each of src and dst is either device memory
 * or pinned host memory (see above), 16-byte aligned, in place (src == dst)
 * or not overlapping.  `mode` is an ms_host_mode.  Stream-ordered on
 * `stream` (NULL = the context's stream): the work starts after what is
 * already enqueued there, and work enqueued there afterwards, including a
 * stream synchronization before the host reads dst, starts after it.
 * Returns once enqueued; n_pages == 0 is a no-op.  The staged modes use the
 * context's staging buffers (host_chunk_pages x host_stage_slots pages of
 * device memory, allocated on the first staged call and wiped at
 * ms_shutdown); concurrent staged calls are serialized.  Errors: MS_EINVAL
 * (size, alignment, overlap, unpinned or out-of-range buffer, bad mode),
 * MS_ENOKEY, MS_ENOMEM (staging), MS_EDEVICE.
 */
ms_status ms_encrypt_host_pages(ms_ctx *ctx, ms_key key, const void *src,
                                void *dst, uint64_t n_pages,
                                const ms_nonce *nonce, int32_t mode,
                                void *stream);
ms_status ms_decrypt_host_pages(ms_ctx *ctx, ms_key key, const void *src,
                                void *dst, uint64_t n_pages,
                                const ms_nonce *nonce, int32_t mode,
                                void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_HOST_H */
