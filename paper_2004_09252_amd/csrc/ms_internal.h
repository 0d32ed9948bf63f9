// Hooks into the engine context (engine.cpp) for the library's other host
// sources.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "memshield.h"
#include "memshield_resident.h"

struct HostPath;  // host-resident page state, defined in host_pages.cpp

int ms_internal_device(ms_ctx* c);
int ms_internal_cu_count(ms_ctx* c);
const ms_config& ms_internal_config(ms_ctx* c);
// The caller's stream, or the context's stream for NULL.
hipStream_t ms_internal_stream(ms_ctx* c, void* stream);
// A device range [p, p+bytes) inside one allocation of the context's device.
ms_status ms_internal_check_range(ms_ctx* c, const void* p, uint64_t bytes,
                                  uint64_t align);
// Maps a HIP error to MS_EDEVICE and makes it sticky.
ms_status ms_internal_dev_err(ms_ctx* c, hipError_t e);
// MS_EDEVICE once a device error has been seen, MS_OK otherwise.
ms_status ms_internal_sticky(ms_ctx* c);
// Key handle -> key-table row; false for an unknown or stale handle.
bool ms_internal_resolve_key(ms_ctx* c, ms_key key, uint32_t* slot);
// Resolve and pin a key handle for a synchronous call: until the matching
// unpin, ms_key_destroy of that handle returns MS_EBUSY.  Unpin once the
// call's launches are enqueued.  MS_ENOKEY for an unknown or stale handle.
ms_status ms_internal_pin_key(ms_ctx* c, ms_key key, uint32_t* slot);
void ms_internal_unpin_key(ms_ctx* c, uint32_t slot);
// One plain launch (split where a launch would exceed its page limit) of
// n_pages pages from src to dst, both GPU-visible addresses, page p taking
// the nonce of page p of `nonce`, with at most `max_waves` waves (0 = as
// many as stay resident).  No argument checks.
ms_status ms_internal_launch_plain(ms_ctx* c, uint32_t key_slot,
                                   const void* src, void* dst,
                                   uint64_t n_pages, const ms_nonce& nonce,
                                   hipStream_t stream, uint32_t max_waves = 0);

// Owned by host_pages.cpp: created by ms_init, destroyed by ms_shutdown
// after the device is idle.
HostPath* ms_internal_host_path_create();
void ms_internal_host_path_destroy(HostPath* h);
HostPath* ms_internal_host_path(ms_ctx* c);

// [p, p+bytes) in pinned host memory mapped into the GPU's address space
// (checked against its allocation when pointer validation is on); *gpu gets
// the address the GPU uses for p.  MS_EINVAL for anything else.
ms_status ms_internal_classify_host(ms_ctx* c, const void* p, uint64_t bytes,
                                    uint64_t align, uint64_t* gpu);
// The same, but [p, p+bytes) may also be device memory of the context's GPU
// (then *gpu = p).
ms_status ms_internal_classify_any(ms_ctx* c, const void* p, uint64_t bytes,
                                   uint64_t align, uint64_t* gpu);

// Copies the 32 key bytes of `key` from the key table into device memory at
// `dst` (device to device, on `stream`, waited for), under the key lock so
// the key cannot be destroyed meanwhile.  MS_ENOKEY for an unknown handle.
ms_status ms_internal_copy_key(ms_ctx* c, ms_key key, void* dst,
                               hipStream_t stream);

// Stops every resident-key engine of the context (resident.cpp).
void ms_internal_resident_stop_all(ms_ctx* c);

// The ring of the context's serving stage (resident.cpp): a resident kernel
// that holds no key of its own and reads, for each descriptor, the row of
// the context's device key table (`key_table`, `table_rows` rows) the
// descriptor names.  Not registered with the context: its owner stops it
// with ms_internal_ring_stop.  It runs the context's cipher and rounds.
ms_status ms_internal_ring_start(ms_ctx* c, const ms_resident_config* cfg,
                                 const uint32_t* key_table,
                                 uint32_t table_rows, ms_resident** out);
// Publish one request (device pages, already validated) with key-table row
// `key_row`; MS_EAGAIN while the ring slots it needs are busy, MS_ECLOSED
// once the kernel has ended, MS_EDEVICE after a descriptor error.  The
// ticket is polled with ms_resident_poll.
ms_status ms_internal_ring_publish(ms_resident* r, uint32_t key_row,
                                   const void* src, void* dst,
                                   uint64_t n_pages, const ms_nonce& nonce,
                                   ms_ticket* ticket_out);
// 1 once every position of a ring ticket has completed, else 0.
int ms_internal_ring_done(ms_resident* r, ms_ticket t);
// The ring positions [first, first + count) a ring ticket holds.
void ms_internal_ring_span(ms_ticket t, uint64_t* first, uint64_t* count);
// Positions handed out so far (every position below it has been published).
uint64_t ms_internal_ring_published(ms_resident* r);
// The first position p in [from, limit) whose completion word does not yet
// say done (limit if there is none): with `from` a completed prefix of the
// ring, the longer prefix, one read per position it passes.
uint64_t ms_internal_ring_advance(ms_resident* r, uint64_t from,
                                  uint64_t limit);
bool ms_internal_ring_alive(ms_resident* r);
// Resident kernels of this process running on `device` (any context's
// engines and serving rings); each holds one wave on every SIMD of the
// compute units it spans.
uint32_t ms_internal_resident_live(int device);
void ms_internal_ring_stop(ms_resident* r);
