// ChaCha page-cipher kernels for gfx950 (CDNA4).
//
// What is computed (MemShield, section 4.4): a 4096-byte page is XORed with
// 64 keystream blocks of 64 bytes; block j of a page comes from ChaCha (20
// rounds unless a reduced-round variant is asked for) on the state
//   [ sigma0..3 | key0..7 | j | nonce0..2 ]
// with the block counter j = 0..63 equal to the block's index in the page;
// encryption and decryption are the same XOR.
//
// Mapping to the hardware (the paper used one 32-thread warp per page, two
// blocks per thread, on a 2014 GPU; this design is for 64-lane CDNA4):
//   * one wavefront owns one page at a time and lane j computes keystream
//     block j, so key and nonce are wave-uniform and sit in SGPRs and the
//     counter is the lane id;
//   * the part of the first double round that does not depend on the
//     counter (three of the four column quarter rounds, and the start of two
//     diagonal ones) is the same for every lane: it runs once per page on the
//     scalar unit instead of 64 times on the vector unit, which removes about
//     4% of the vector instructions; the 16 state words stay in VGPRs and each
//     add, xor and rotate is one 32-bit vector instruction (rotates are
//     v_alignbit_b32);
//   * global memory is read and written fully coalesced (a wave's dwordx4
//     access covers 1 KiB of consecutive bytes) with non-temporal hints,
//     because the data is touched once; the keystream, produced in block
//     order per lane, is turned into that consecutive order through a 4 KiB
//     per-wave LDS buffer (write by block, read by 16-byte column, XOR-swizzled
//     so neither side conflicts on LDS banks);
//   * waves are persistent over pages: each wave walks its pages with the
//     next page's loads in flight while the current page is ciphered
//     ("unroll" 2), or one page at a time ("unroll" 1);
//   * no matrix cores: the keystream is integer ALU work.
//
// The same kernels run a second cipher, Salsa20 (ChaCha's predecessor, the
// paper's replaceable cipher of sections 1 and 6), chosen per context:
// words 6, 7 of its state take the page nonce's words 0, 1, its 64-bit
// block counter is (page nonce word 2, j); see cipher_core.h.
//
// The plain kernel takes one run of pages with one key and one nonce rule.
// The batched kernel walks a flattened list of (request, page) items, each
// request with its own key slot and nonce rule, taking `pages_per_wave`
// consecutive items at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cipher_core.h"
#include "ms_kernels.h"

namespace ms {
namespace {
// ---------------------------------------------------------------- plain ---

// Pages first_page + w, + W, + 2W, ... of the caller's run for wave w of W.
// The launch arguments are copied in by value so that every field stays a
// scalar (wave-uniform) value; page counters are 32-bit (one launch covers
// at most 2^24 pages) so that loop tests stay on the scalar unit.
template <uint32_t KIND>
struct PlainPages {
  const uint8_t* src;
  uint8_t* dst;
  const uint32_t* nonce_array;
  uint64_t nonce_base;
  uint64_t nonce_stride;
  uint64_t first_page;
  const uint32_t* keys;
  uint32_t n_pages;
  uint32_t nonce_tag;
  uint32_t key_slot;
  uint32_t page;   // next page index within this launch
  uint32_t step;

  __device__ __forceinline__ bool next(PageJob& j) {
    if (page >= n_pages) return false;
    const uint64_t p = first_page + page;
    page += step;
    j.src = reinterpret_cast<const uint4*>(src + p * kPageBytes);
    j.dst = reinterpret_cast<uint4*>(dst + p * kPageBytes);
    j.slot = key_slot;
    if (KIND == kNonceArray) {
      const auto* n = cnst(nonce_array) + p * 3u;
      j.n[0] = n[0];
      j.n[1] = n[1];
      j.n[2] = n[2];
    } else {
      const uint64_t v = nonce_base + p * nonce_stride;
      j.n[0] = (uint32_t)v;
      j.n[1] = (uint32_t)(v >> 32);
      j.n[2] = nonce_tag;
    }
    return true;
  }

  // The key is re-read (one scalar load, scalar-cache hit) for every page
  // rather than kept live across the loop.
  __device__ __forceinline__ void key(const PageJob& j, uint32_t (&out)[8]) {
    uint32_t slot = uni(j.slot);
    asm volatile("" : "+s"(slot));
    const auto* kp = cnst(keys) + (uint64_t)slot * 8u;
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = kp[i];
  }
};

template <uint32_t CIPHER, int ROUNDS, int UNROLL, uint32_t KIND>
__global__ __launch_bounds__(kBlockThreads, UNROLL == 2 ? 7 : 8) void plain_pages_kernel(
    PlainArgs a) {
  __shared__ uint4 lds[kWavesPerBlock][256];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t w = wave_in_block();
  PlainPages<KIND> src;
  src.src = a.src;
  src.dst = a.dst;
  src.nonce_array = a.nonce_array;
  src.nonce_base = a.nonce_base;
  src.nonce_stride = a.nonce_stride;
  src.first_page = a.first_page;
  src.n_pages = (uint32_t)a.n_pages;
  src.nonce_tag = a.nonce_tag;
  src.keys = a.keys;
  src.key_slot = a.key_slot;
  src.page = blockIdx.x * kWavesPerBlock + w;
  src.step = gridDim.x * kWavesPerBlock;
  run_pages<ROUNDS, UNROLL, CIPHER>(src, lds[w], lane);
}

// -------------------------------------------------------------- batched ---

// The wave's items are chunks c = wave, wave + W, ... of pages_per_wave
// consecutive pages in the batch's flattened page space.
struct BatchPages {
  const DevReq* reqs;
  const uint32_t* keys;
  uint64_t total;
  uint32_t n_req;
  uint32_t ppw;
  uint64_t chunk_step;   // W * ppw
  uint64_t p;            // next page
  uint64_t chunk_end;    // end of the current chunk
  uint32_t r;            // request holding page p (valid inside a chunk)

  __device__ __forceinline__ void start_chunk(uint64_t c0) {
    p = c0;
    chunk_end = min(c0 + ppw, total);
    // last request whose first page is <= c0 (page_begin increases)
    uint32_t lo = 0, hi = n_req;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (cnst(reqs)[mid].page_begin <= c0) lo = mid; else hi = mid;
    }
    r = lo;
  }

  __device__ __forceinline__ bool next(PageJob& j) {
    if (p >= chunk_end) return false;
    const auto* rq = cnst(reqs);
    while (rq[r].page_end <= p) ++r;
    const auto* q = rq + r;
    const uint64_t i = p - q->page_begin;
    j.src = reinterpret_cast<const uint4*>(q->src + i * kPageBytes);
    j.dst = reinterpret_cast<uint4*>(q->dst + i * kPageBytes);
    j.slot = q->key_slot;
    if (q->kind == kNonceArray) {
      const auto* n =
          cnst(reinterpret_cast<const uint32_t*>(q->nonce)) + i * 3u;
      j.n[0] = n[0];
      j.n[1] = n[1];
      j.n[2] = n[2];
    } else {
      const uint64_t v = q->nonce + i * q->stride;
      j.n[0] = (uint32_t)v;
      j.n[1] = (uint32_t)(v >> 32);
      j.n[2] = q->tag;
    }
    ++p;
    return true;
  }

  __device__ __forceinline__ void key(const PageJob& j, uint32_t (&out)[8]) {
    uint32_t slot = uni(j.slot);
    asm volatile("" : "+s"(slot));
    const auto* kp = cnst(keys) + (uint64_t)slot * 8u;
#pragma unroll
    for (int t = 0; t < 8; ++t) out[t] = kp[t];
  }
};

// Chains the wave's chunks into one page stream for run_pages.
struct BatchStream {
  BatchPages b;
  uint64_t c0;   // first page of the current chunk

  __device__ __forceinline__ bool next(PageJob& j) {
    for (;;) {
      if (c0 >= b.total) return false;
      if (b.next(j)) return true;
      c0 += b.chunk_step;
      if (c0 >= b.total) return false;
      b.start_chunk(c0);
    }
  }

  __device__ __forceinline__ void key(const PageJob& j, uint32_t (&out)[8]) {
    b.key(j, out);
  }
};

template <uint32_t CIPHER, int ROUNDS, int UNROLL>
__device__ __forceinline__ void batch_body(const DevBatchHdr* hdr,
                                           const DevReq* reqs,
                                           const uint32_t* keys,
                                           uint32_t pages_per_wave,
                                           uint4* lds, uint32_t w) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = (uint64_t)blockIdx.x * kWavesPerBlock + w;
  BatchStream s;
  s.b.reqs = reqs;
  s.b.keys = keys;
  s.b.total = cnst(hdr)->total_pages;
  s.b.n_req = cnst(hdr)->n_req;
  s.b.ppw = pages_per_wave;
  s.b.chunk_step = (uint64_t)gridDim.x * kWavesPerBlock * pages_per_wave;
  s.c0 = wave * pages_per_wave;
  if (s.c0 >= s.b.total) return;
  s.b.start_chunk(s.c0);
  run_pages<ROUNDS, UNROLL, CIPHER>(s, lds, lane);
}

// Descriptors in device memory (copied there before the launch).
template <uint32_t CIPHER, int ROUNDS, int UNROLL>
__global__ __launch_bounds__(kBlockThreads, UNROLL == 2 ? 7 : 8) void batch_pages_kernel(
    const DevBatchHdr* __restrict__ hdr, const uint32_t* __restrict__ keys,
    uint32_t pages_per_wave) {
  __shared__ uint4 lds[kWavesPerBlock][256];
  const uint32_t w = wave_in_block();
  batch_body<CIPHER, ROUNDS, UNROLL>(
      hdr, reinterpret_cast<const DevReq*>(hdr + 1), keys, pages_per_wave,
      lds[w], w);
}

// The same batch with its header and records in the kernel arguments (a
// batch of at most kInlineBatchMax requests), so that no descriptor copy has
// to run before it.  They are read where the dispatch placed the arguments,
// through the kernarg segment pointer, with scalar loads like the device
// array of the kernel above.
template <uint32_t CIPHER, int ROUNDS, int UNROLL>
__global__ __launch_bounds__(kBlockThreads, UNROLL == 2 ? 7 : 8) void batch_inline_kernel(
    InlineBatch batch, const uint32_t* __restrict__ keys,
    uint32_t pages_per_wave) {
  (void)batch;
  __shared__ uint4 lds[kWavesPerBlock][256];
  const uint32_t w = wave_in_block();
  const auto* kb = (const __attribute__((address_space(4))) InlineBatch*)
      __builtin_amdgcn_kernarg_segment_ptr();
  batch_body<CIPHER, ROUNDS, UNROLL>(
      (const DevBatchHdr*)&kb->hdr, (const DevReq*)&kb->req[0], keys,
      pages_per_wave, lds[w], w);
}

// --------------------------------------------------------------- probes ---

// Streaming copy: one wave per 4 KiB page, coalesced non-temporal dwordx4
// accesses, the same memory pattern as the page kernels without arithmetic.
__global__ __launch_bounds__(kBlockThreads) void copy_probe_kernel(
    const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n16) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t chunk =
      (uint64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const uint64_t base = chunk * 256;
  if (base + 256 <= n16) {
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = load_nt(src + base + q * 64 + lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) store_nt(v[q], dst + base + q * 64 + lane);
  } else {
    for (uint64_t i = base + lane; i < n16; i += kWave) dst[i] = src[i];
  }
}

constexpr int kValuChains = 8;
constexpr int kValuUnroll = 4;

// Integer VALU throughput: 8 independent chains of (xor, rotate, add), the
// three operation kinds of the cipher, all lane-varying.
__global__ __launch_bounds__(kBlockThreads) void valu_probe_kernel(
    uint32_t* __restrict__ out, uint32_t iters) {
  uint32_t x[kValuChains], y[kValuChains];
  const uint32_t gid = blockIdx.x * kBlockThreads + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kValuChains; ++c) {
    x[c] = gid * (2u * c + 1u);
    y[c] = gid ^ (0x9e3779b9u * (c + 1u));
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kValuUnroll; ++k) {
#pragma unroll
      for (int c = 0; c < kValuChains; ++c) {
        x[c] = rotl32(x[c] ^ y[c], 7);
        y[c] += x[c];
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kValuChains; ++c) acc ^= x[c] + y[c];
  out[gid] = acc;
}

__global__ __launch_bounds__(kBlockThreads) void fill_u32_kernel(
    uint32_t* __restrict__ dst, uint32_t value, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlockThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < n;
       i += stride)
    dst[i] = value;
}

// A batch's request records, from the pinned host staging buffer into the
// device array the batch kernel reads.  It runs on the batch's own queue, so
// the batch kernel waits for it by queue order alone; a copy-engine transfer
// would add a wait across engines before and after it.  The loads are
// system-scope, so they read what the host wrote before the launch.
__global__ __launch_bounds__(kBlockThreads) void desc_copy_kernel(
    uint4* __restrict__ dst, const uint64_t* __restrict__ src, uint32_t n16) {
  const uint32_t i = blockIdx.x * kBlockThreads + threadIdx.x;
  if (i >= n16) return;
  const uint64_t lo =
      __hip_atomic_load(src + 2u * i, __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_SYSTEM);
  const uint64_t hi =
      __hip_atomic_load(src + 2u * i + 1u, __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_SYSTEM);
  dst[i] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi,
                      (uint32_t)(hi >> 32));
}

// Plain kernel for one (cipher, rounds, unroll, nonce kind).
template <uint32_t CIPHER, int ROUNDS, int UNROLL>
const void* plain_fn(uint32_t kind) {
  return kind == kNonceArray
             ? reinterpret_cast<const void*>(
                   &plain_pages_kernel<CIPHER, ROUNDS, UNROLL, kNonceArray>)
             : reinterpret_cast<const void*>(
                   &plain_pages_kernel<CIPHER, ROUNDS, UNROLL, kNonceLinear>);
}

template <uint32_t CIPHER>
const void* plain_fn_c(uint32_t unroll, int rounds, uint32_t kind) {
  if (unroll == 2) {
    switch (rounds) {
      case 20: return plain_fn<CIPHER, 20, 2>(kind);
      case 12: return plain_fn<CIPHER, 12, 2>(kind);
      case 8: return plain_fn<CIPHER, 8, 2>(kind);
    }
  } else if (unroll == 1) {
    switch (rounds) {
      case 20: return plain_fn<CIPHER, 20, 1>(kind);
      case 12: return plain_fn<CIPHER, 12, 1>(kind);
      case 8: return plain_fn<CIPHER, 8, 1>(kind);
    }
  }
  return nullptr;
}

template <uint32_t CIPHER>
const void* batch_fn_c(uint32_t unroll, int rounds) {
#define MS_BATCH_FN(R, U) \
  reinterpret_cast<const void*>(&batch_pages_kernel<CIPHER, R, U>)
  if (unroll == 2) {
    switch (rounds) {
      case 20: return MS_BATCH_FN(20, 2);
      case 12: return MS_BATCH_FN(12, 2);
      case 8: return MS_BATCH_FN(8, 2);
    }
  } else if (unroll == 1) {
    switch (rounds) {
      case 20: return MS_BATCH_FN(20, 1);
      case 12: return MS_BATCH_FN(12, 1);
      case 8: return MS_BATCH_FN(8, 1);
    }
  }
#undef MS_BATCH_FN
  return nullptr;
}

template <uint32_t CIPHER>
const void* batch_inline_fn_c(uint32_t unroll, int rounds) {
#define MS_INLINE_FN(R, U) \
  reinterpret_cast<const void*>(&batch_inline_kernel<CIPHER, R, U>)
  if (unroll == 2) {
    switch (rounds) {
      case 20: return MS_INLINE_FN(20, 2);
      case 12: return MS_INLINE_FN(12, 2);
      case 8: return MS_INLINE_FN(8, 2);
    }
  } else if (unroll == 1) {
    switch (rounds) {
      case 20: return MS_INLINE_FN(20, 1);
      case 12: return MS_INLINE_FN(12, 1);
      case 8: return MS_INLINE_FN(8, 1);
    }
  }
#undef MS_INLINE_FN
  return nullptr;
}

}  // namespace

const void* plain_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds,
                            uint32_t kind) {
  switch (cipher) {
    case kCipherChaCha: return plain_fn_c<kCipherChaCha>(unroll, rounds, kind);
    case kCipherSalsa: return plain_fn_c<kCipherSalsa>(unroll, rounds, kind);
  }
  return nullptr;
}

const void* batch_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds) {
  switch (cipher) {
    case kCipherChaCha: return batch_fn_c<kCipherChaCha>(unroll, rounds);
    case kCipherSalsa: return batch_fn_c<kCipherSalsa>(unroll, rounds);
  }
  return nullptr;
}

hipError_t launch_batch_inline(const InlineBatch& batch, const uint32_t* keys,
                               uint32_t pages_per_wave, uint32_t unroll,
                               uint32_t grid_blocks, uint32_t cipher,
                               int rounds, hipStream_t stream) {
  const void* fn = nullptr;
  switch (cipher) {
    case kCipherChaCha:
      fn = batch_inline_fn_c<kCipherChaCha>(unroll, rounds);
      break;
    case kCipherSalsa:
      fn = batch_inline_fn_c<kCipherSalsa>(unroll, rounds);
      break;
  }
  if (!fn || pages_per_wave == 0 || grid_blocks == 0 ||
      batch.hdr.n_req == 0 || batch.hdr.n_req > kInlineBatchMax)
    return hipErrorInvalidValue;
  // the runtime copies the arguments at the launch
  void* args[] = {const_cast<InlineBatch*>(&batch), (void*)&keys,
                  (void*)&pages_per_wave};
  return hipLaunchKernel(fn, dim3(grid_blocks), dim3(kBlockThreads), args, 0,
                         stream);
}

hipError_t launch_plain(const PlainArgs& a, uint32_t kind, uint32_t cipher,
                        int rounds, uint32_t max_waves, uint32_t unroll,
                        hipStream_t stream) {
  const void* fn = plain_kernel_fn(unroll, cipher, rounds, kind);
  if (!fn || max_waves == 0) return hipErrorInvalidValue;
  for (uint64_t done = 0; done < a.n_pages;) {
    PlainArgs part = a;
    part.first_page = a.first_page + done;
    part.n_pages = a.n_pages - done;
    if (part.n_pages > kMaxPagesPerPlainLaunch)
      part.n_pages = kMaxPagesPerPlainLaunch;
    // one wave per page up to max_waves waves; beyond that waves loop
    const uint64_t waves = part.n_pages < max_waves ? part.n_pages : max_waves;
    const uint32_t grid =
        (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    void* args[] = {(void*)&part};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kBlockThreads),
                                         args, 0, stream);
    if (e != hipSuccess) return e;
    done += part.n_pages;
  }
  return hipSuccess;
}

uint32_t resident_waves_per_cu(const void* fn) {
  int blocks = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &blocks, fn, kBlockThreads, 0) != hipSuccess ||
      blocks <= 0)
    return 0;
  return (uint32_t)blocks * kWavesPerBlock;
}

hipError_t launch_batch(const DevBatchHdr* batch, const uint32_t* keys,
                        uint32_t pages_per_wave, uint32_t unroll,
                        uint32_t grid_blocks, uint32_t cipher, int rounds,
                        hipStream_t stream) {
  const void* fn = batch_kernel_fn(unroll, cipher, rounds);
  if (!fn || pages_per_wave == 0 || grid_blocks == 0)
    return hipErrorInvalidValue;
  void* args[] = {(void*)&batch, (void*)&keys, (void*)&pages_per_wave};
  return hipLaunchKernel(fn, dim3(grid_blocks), dim3(kBlockThreads), args, 0,
                         stream);
}

const void* desc_copy_fn() {
  return reinterpret_cast<const void*>(&desc_copy_kernel);
}

uint32_t desc_copy_blocks(size_t bytes) {
  const size_t n16 = bytes / 16;
  return (uint32_t)((n16 + kBlockThreads - 1) / kBlockThreads);
}

hipError_t launch_desc_copy(void* dev, const void* host, size_t bytes,
                            hipStream_t stream) {
  if (!dev || !host || bytes == 0 || bytes % 16 != 0 ||
      bytes / 16 > 0xffffffffull)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(desc_copy_kernel, dim3(desc_copy_blocks(bytes)),
                     dim3(kBlockThreads), 0, stream,
                     reinterpret_cast<uint4*>(dev),
                     reinterpret_cast<const uint64_t*>(host),
                     (uint32_t)(bytes / 16));
  return hipGetLastError();
}

// Request descriptors of ms_process_batch_static.  Host code must not pass
// this name to a kernel or a copy: on the host it only stands for the
// symbol; its device address comes from static_batch_scratch.
static __device__ __align__(256) uint8_t scratch[kStaticBatchBytes];

hipError_t static_batch_scratch(void** out) {
  if (!out) return hipErrorInvalidValue;
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes,
                       uint32_t grid_blocks, hipStream_t stream) {
  (void)grid_blocks;  // one wave per 4 KiB chunk
  if (bytes % 16 != 0) return hipErrorInvalidValue;
  const uint64_t n16 = bytes / 16;
  const uint64_t chunks = (n16 + 255) / 256;
  const uint64_t blocks = (chunks + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks == 0 || blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_probe_kernel, dim3((uint32_t)blocks),
                     dim3(kBlockThreads), 0, stream,
                     reinterpret_cast<const uint4*>(src),
                     reinterpret_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_valu(uint32_t* out, uint32_t iters, uint32_t grid_blocks,
                       hipStream_t stream) {
  if (grid_blocks == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(valu_probe_kernel, dim3(grid_blocks), dim3(kBlockThreads),
                     0, stream, out, iters);
  return hipGetLastError();
}

uint64_t valu_probe_ops(uint32_t iters, uint32_t grid_blocks) {
  // per thread and iteration: chains x unroll x (xor + rotate + add)
  return (uint64_t)iters * kValuChains * kValuUnroll * 3ull *
         (uint64_t)grid_blocks * kBlockThreads;
}

hipError_t launch_fill_u32(uint32_t* dst, uint32_t value, uint64_t n_words,
                           hipStream_t stream) {
  if (n_words == 0) return hipSuccess;
  uint64_t blocks = (n_words + kBlockThreads - 1) / kBlockThreads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks),
                     dim3(kBlockThreads), 0, stream, dst, value, n_words);
  return hipGetLastError();
}

}  // namespace ms
