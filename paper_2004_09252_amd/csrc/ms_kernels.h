// Internal interface between the engine (engine.cpp) and the gfx950 kernels
// (page_cipher.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

constexpr uint32_t kPageBytes = 4096;
constexpr uint32_t kWave = 64;           // CDNA wavefront width
constexpr uint32_t kBlockThreads = 256;  // 4 waves per workgroup
constexpr uint32_t kWavesPerBlock = kBlockThreads / kWave;

enum NonceKind : uint32_t { kNonceArray = 0, kNonceLinear = 1 };

// Stream cipher of the page kernels (the values of ms_config.cipher).
enum CipherKind : uint32_t { kCipherChaCha = 0, kCipherSalsa = 1 };

// One request of a fused batch, as the batch kernel reads it from device
// memory.  64 bytes, so a wave fetches one with scalar loads.
struct DevReq {
  uint64_t src;         // device address of the request's first source page
  uint64_t dst;         // device address of its first destination page
  uint64_t nonce;       // kNonceArray: device address of 12-byte nonces;
                        // kNonceLinear: nonce base
  uint64_t stride;      // kNonceLinear: nonce increment per page
  uint64_t page_begin;  // first page of this request in the batch's
                        // flattened page space
  uint64_t page_end;    // one past its last page (page_begin < page_end)
  uint32_t key_slot;    // row of the device key table
  uint32_t kind;        // NonceKind
  uint32_t tag;         // kNonceLinear: word 15 of the cipher state
  uint32_t pad;
};
static_assert(sizeof(DevReq) == 64, "DevReq layout");

// Header of a batch buffer; DevReq[n_req] follows it directly.
struct DevBatchHdr {
  uint64_t total_pages;  // == last request's page_end
  uint32_t n_req;
  uint32_t pad0;
  uint64_t pad[6];
};
static_assert(sizeof(DevBatchHdr) == 64, "DevBatchHdr layout");

// A batch of at most kInlineBatchMax requests whose header and records
// travel in the kernel arguments (no descriptor copy before the launch).
constexpr uint32_t kInlineBatchMax = 15;
struct InlineBatch {
  DevBatchHdr hdr;
  DevReq req[kInlineBatchMax];
};
static_assert(sizeof(InlineBatch) == 64 * (1 + kInlineBatchMax),
              "InlineBatch layout");

// Arguments of one plain launch over a run of pages.
struct PlainArgs {
  const uint32_t* keys;  // device key table, 8 words per slot
  const uint8_t* src;
  uint8_t* dst;
  const uint32_t* nonce_array;  // kNonceArray: 3 words per page
  uint64_t nonce_base;
  uint64_t nonce_stride;
  uint64_t first_page;   // pages [first_page, first_page + n_pages) of the run
  uint64_t n_pages;
  uint32_t key_slot;
  uint32_t nonce_tag;
};

// All launchers return the HIP status of the launch.
// Plain launch: one wave per page up to `max_waves` waves, which then loop
// over the remaining pages; `unroll` 2 overlaps a page's loads with the
// previous page's cipher work, 1 does not.
// `cipher` is a CipherKind, `rounds` 20, 12 or 8.
hipError_t launch_plain(const PlainArgs& a, uint32_t kind, uint32_t cipher,
                        int rounds, uint32_t max_waves, uint32_t unroll,
                        hipStream_t stream);
hipError_t launch_batch(const DevBatchHdr* batch, const uint32_t* keys,
                        uint32_t pages_per_wave, uint32_t unroll,
                        uint32_t grid_blocks, uint32_t cipher, int rounds,
                        hipStream_t stream);
// The fused batch kernel reading its records from the kernel arguments.
hipError_t launch_batch_inline(const InlineBatch& batch, const uint32_t* keys,
                               uint32_t pages_per_wave, uint32_t unroll,
                               uint32_t grid_blocks, uint32_t cipher,
                               int rounds, hipStream_t stream);
// Kernel entry points (graph capture, occupancy queries); nullptr for a
// combination that does not exist.
const void* batch_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds);
const void* plain_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds,
                            uint32_t kind);
// Copies a batch buffer of `bytes` (a multiple of 16) from pinned host
// memory `host` to device memory `dev` with a kernel on `stream` (see
// desc_copy_kernel); desc_copy_fn and desc_copy_blocks give its entry point
// and grid for graph kernel nodes (arguments: dev, host, bytes / 16).
hipError_t launch_desc_copy(void* dev, const void* host, size_t bytes,
                            hipStream_t stream);
const void* desc_copy_fn();
uint32_t desc_copy_blocks(size_t bytes);
// A plain launch covers at most this many pages (32-bit page counters in
// the kernel); longer runs are split into several launches.
constexpr uint64_t kMaxPagesPerPlainLaunch = 1ull << 24;
// Waves of `fn` (256-thread workgroups) that fit on one compute unit at once;
// 0 if the runtime cannot say.
uint32_t resident_waves_per_cu(const void* fn);

// Descriptor array of ms_process_batch_static: one batch header and up to
// kStaticBatchMaxRequests request records, a file-scope device array in
// page_cipher.hip (one copy per device, for the life of the process).
constexpr uint32_t kStaticBatchMaxRequests = 4096;
constexpr size_t kStaticBatchBytes =
    sizeof(DevBatchHdr) + (size_t)kStaticBatchMaxRequests * sizeof(DevReq);
// The current device's address of that array (hipGetSymbolAddress).
hipError_t static_batch_scratch(void** out);

// Calibration probes.
hipError_t launch_copy(const void* src, void* dst, uint64_t bytes,
                       uint32_t grid_blocks, hipStream_t stream);
hipError_t launch_valu(uint32_t* out, uint32_t iters, uint32_t grid_blocks,
                       hipStream_t stream);
// Independent 32-bit VALU operations one launch of launch_valu performs.
uint64_t valu_probe_ops(uint32_t iters, uint32_t grid_blocks);
// Fill kernel (used instead of memset where a graph may capture it).
hipError_t launch_fill_u32(uint32_t* dst, uint32_t value, uint64_t n_words,
                           hipStream_t stream);

}  // namespace ms
