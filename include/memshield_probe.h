/*
 * memshield_probe.h - calibration probes of the page-cipher engine.
 *
 * The page cipher is bound by 32-bit integer ALU throughput with HBM close
 * behind (a ChaCha20 page costs about 15.5 integer operations per byte and
 * moves 2 bytes of HBM traffic per byte).  These two kernels measure the
 * ceilings the cipher kernels are compared against on the running device:
 *   - a streaming dwordx4 copy (read + write, no arithmetic): the HBM rate
 *     the page kernels' own access pattern can reach, and the reference
 *     byte count for scaling hardware traffic counters;
 *   - an integer VALU kernel of independent xor / rotate / add chains (the
 *     cipher's three operations), no memory traffic: the sustained integer
 *     operation rate.
 * Both are stream-ordered and return once enqueued; pointers are device
 * memory owned by the caller and checked like the cipher calls' pointers.
 */
#ifndef MEMSHIELD_PROBE_H
#define MEMSHIELD_PROBE_H

#include "memshield.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Copy `bytes` (multiple of 16) from src to dst (device, 16-byte aligned, not
 * overlapping) with `grid_blocks` workgroups of 256 threads (0 = 8 per
 * compute unit).  Errors: MS_EINVAL, MS_EDEVICE.
 */
ms_status ms_probe_copy(ms_ctx *ctx, const void *src, void *dst,
                        uint64_t bytes, uint32_t grid_blocks, void *stream);

/*
 * Run `iters` iterations of the integer chains in `grid_blocks` workgroups of
 * 256 threads (0 = 32 per compute unit), writing one word per thread to `out`
 * (device, grid_blocks*256*4 bytes).  *ops_out (may be NULL) receives the
 * number of 32-bit VALU operations the launch performs.
 */
ms_status ms_probe_valu(ms_ctx *ctx, uint32_t *out, uint32_t iters,
                        uint32_t grid_blocks, void *stream, uint64_t *ops_out);

/*
 * Host-link probe: move `bytes` (multiple of 16) from src to dst, where each
 * side is device memory or pinned host memory (as for the calls of
 * memshield_host.h), not overlapping.  engine 0: the copy kernel above, which
 * reads and writes host memory through the link directly (the path of
 * MS_HOST_MAPPED); engine 1: the copy engines (hipMemcpyAsync, the path of
 * MS_HOST_DMA).  Host-to-device, device-to-host, and both at once on two
 * streams give the link rates the host-page calls are compared against.
 * Stream-ordered.  Errors: MS_EINVAL, MS_EDEVICE.
 */
ms_status ms_probe_link(ms_ctx *ctx, const void *src, void *dst,
                        uint64_t bytes, int32_t engine, void *stream);

/* Compute units of the context's device (the grid sizing unit above). */
int ms_device_cu_count(ms_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MEMSHIELD_PROBE_H */
