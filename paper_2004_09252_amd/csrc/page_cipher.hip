// ChaCha page-cipher kernels for gfx950 (CDNA4).
//
// What is computed (MemShield, section 4.4): a 4096-byte page is XORed with
// 64 keystream blocks of 64 bytes; block j of a page comes from ChaCha (20
// rounds unless a reduced-round variant is asked for) on the state
//   [ sigma0..3 | key0..7 | j | nonce0..2 ]
// with the block counter j = 0..63 equal to the block's index in the page;
// encryption and decryption are the same XOR.
//
// Mapping to the hardware (differs from the paper's one-warp-per-page,
// two-blocks-per-thread design for its 32-wide GPU):
//   * one 64-lane wavefront owns a page and lane j computes block j, so the
//     key and nonce are wave-uniform and live in SGPRs, the counter is the
//     lane id, and all of the first column round except the column that
//     holds the counter is uniform work the compiler moves to the scalar
//     unit;
//   * the 16 state words stay in VGPRs for all rounds; each add, xor and
//     rotate is one 32-bit VALU instruction (rotates become v_alignbit_b32);
//   * lane j loads and stores its own 64 bytes with four dwordx4 accesses;
//     the four accesses of a wave cover the whole 4 KiB page, so every HBM
//     line is fetched and written once;
//   * no LDS and no matrix cores: the keystream is ALU work and the data
//     never needs to move between lanes.
//
// The batched kernel walks a flattened list of (request, page) items, each
// request with its own key slot and nonce rule, in chunks of
// `pages_per_wave` consecutive pages per wavefront; with UNROLL = 2 a wave
// ciphers two pages at once (two independent blocks per lane) for more
// instruction-level parallelism.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ms_kernels.h"

namespace ms {
namespace {

// "expand 32-byte k" as four little-endian words.
constexpr uint32_t kSigma0 = 0x61707865u;
constexpr uint32_t kSigma1 = 0x3320646eu;
constexpr uint32_t kSigma2 = 0x79622d32u;
constexpr uint32_t kSigma3 = 0x6b206574u;

__device__ __forceinline__ uint32_t rotl32(uint32_t v, uint32_t n) {
  return (v << n) | (v >> (32u - n));
}

// Wave-uniform description of one page: where it is and its key and nonce.
struct PageJob {
  const uint4* src;
  uint4* dst;
  uint32_t k[8];
  uint32_t n[3];
};

// Quarter round (A, B, C, D) applied to U independent states, step by step,
// so that the U dependency chains interleave in the instruction stream.
template <int U, int A, int B, int C, int D>
__device__ __forceinline__ void quarter(uint32_t (&x)[U][16]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][A] += x[u][B];
    x[u][D] = rotl32(x[u][D] ^ x[u][A], 16);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][C] += x[u][D];
    x[u][B] = rotl32(x[u][B] ^ x[u][C], 12);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][A] += x[u][B];
    x[u][D] = rotl32(x[u][D] ^ x[u][A], 8);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][C] += x[u][D];
    x[u][B] = rotl32(x[u][B] ^ x[u][C], 7);
  }
}

// Lane `lane` of the wave XORs block `lane` of each of the U pages.
template <int U, int ROUNDS>
__device__ __forceinline__ void cipher_block_of_pages(const PageJob (&job)[U],
                                                      uint32_t lane) {
  uint4 d[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint4* s = job[u].src + lane * 4u;
#pragma unroll
    for (int q = 0; q < 4; ++q) d[u][q] = s[q];
  }

  uint32_t x[U][16];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][0] = kSigma0;
    x[u][1] = kSigma1;
    x[u][2] = kSigma2;
    x[u][3] = kSigma3;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[u][4 + i] = job[u].k[i];
    x[u][12] = lane;
    x[u][13] = job[u].n[0];
    x[u][14] = job[u].n[1];
    x[u][15] = job[u].n[2];
  }

#pragma unroll
  for (int r = 0; r < ROUNDS; r += 2) {
    quarter<U, 0, 4, 8, 12>(x);
    quarter<U, 1, 5, 9, 13>(x);
    quarter<U, 2, 6, 10, 14>(x);
    quarter<U, 3, 7, 11, 15>(x);
    quarter<U, 0, 5, 10, 15>(x);
    quarter<U, 1, 6, 11, 12>(x);
    quarter<U, 2, 7, 8, 13>(x);
    quarter<U, 3, 4, 9, 14>(x);
  }

#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u][0] += kSigma0;
    x[u][1] += kSigma1;
    x[u][2] += kSigma2;
    x[u][3] += kSigma3;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[u][4 + i] += job[u].k[i];
    x[u][12] += lane;
    x[u][13] += job[u].n[0];
    x[u][14] += job[u].n[1];
    x[u][15] += job[u].n[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      d[u][q].x ^= x[u][4 * q + 0];
      d[u][q].y ^= x[u][4 * q + 1];
      d[u][q].z ^= x[u][4 * q + 2];
      d[u][q].w ^= x[u][4 * q + 3];
    }
    uint4* o = job[u].dst + lane * 4u;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = d[u][q];
  }
}

__device__ __forceinline__ uint32_t wave_in_block() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ void load_key(PageJob& j, const uint32_t* keys,
                                         uint32_t slot) {
  const uint32_t* k = keys + (uint64_t)slot * 8u;
#pragma unroll
  for (int i = 0; i < 8; ++i) j.k[i] = k[i];
}

// ---------------------------------------------------------------- plain ---

template <int ROUNDS, uint32_t KIND>
__global__ __launch_bounds__(kBlockThreads) void plain_pages_kernel(
    PlainArgs a) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t page =
      (uint64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  if (page >= a.n_pages) return;
  const uint64_t p = a.first_page + page;  // index within the caller's run

  PageJob job[1];
  job[0].src = reinterpret_cast<const uint4*>(a.src + p * kPageBytes);
  job[0].dst = reinterpret_cast<uint4*>(a.dst + p * kPageBytes);
  load_key(job[0], a.keys, a.key_slot);
  if (KIND == kNonceArray) {
    const uint32_t* n = a.nonce_array + p * 3u;
    job[0].n[0] = n[0];
    job[0].n[1] = n[1];
    job[0].n[2] = n[2];
  } else {
    const uint64_t v = a.nonce_base + p * a.nonce_stride;
    job[0].n[0] = (uint32_t)v;
    job[0].n[1] = (uint32_t)(v >> 32);
    job[0].n[2] = a.nonce_tag;
  }
  cipher_block_of_pages<1, ROUNDS>(job, lane);
}

// -------------------------------------------------------------- batched ---

__device__ __forceinline__ void job_from_request(PageJob& j, const DevReq* r,
                                                 const uint32_t* keys,
                                                 uint64_t page) {
  const uint64_t i = page - r->page_begin;
  j.src = reinterpret_cast<const uint4*>(r->src + i * kPageBytes);
  j.dst = reinterpret_cast<uint4*>(r->dst + i * kPageBytes);
  load_key(j, keys, r->key_slot);
  if (r->kind == kNonceArray) {
    const uint32_t* n =
        reinterpret_cast<const uint32_t*>(r->nonce) + i * 3u;
    j.n[0] = n[0];
    j.n[1] = n[1];
    j.n[2] = n[2];
  } else {
    const uint64_t v = r->nonce + i * r->stride;
    j.n[0] = (uint32_t)v;
    j.n[1] = (uint32_t)(v >> 32);
    j.n[2] = r->tag;
  }
}

template <int ROUNDS, int UNROLL>
__global__ __launch_bounds__(kBlockThreads) void batch_pages_kernel(
    const DevBatchHdr* __restrict__ hdr, const uint32_t* __restrict__ keys,
    uint32_t pages_per_wave) {
  const DevReq* reqs = reinterpret_cast<const DevReq*>(hdr + 1);
  const uint64_t total = hdr->total_pages;
  const uint32_t n_req = hdr->n_req;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave =
      (uint64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
  const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerBlock;
  const uint64_t step = n_waves * pages_per_wave;

  for (uint64_t c0 = wave * pages_per_wave; c0 < total; c0 += step) {
    const uint64_t c1 = min(c0 + pages_per_wave, total);
    // Last request whose first page is <= c0 (page_begin is increasing).
    uint32_t lo = 0, hi = n_req;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (reqs[mid].page_begin <= c0) lo = mid; else hi = mid;
    }
    uint32_t r = lo;
    uint64_t p = c0;
    if (UNROLL == 2) {
      for (; p + 1 < c1; p += 2) {
        while (reqs[r].page_end <= p) ++r;
        uint32_t r2 = r;
        while (reqs[r2].page_end <= p + 1) ++r2;
        PageJob job[2];
        job_from_request(job[0], reqs + r, keys, p);
        job_from_request(job[1], reqs + r2, keys, p + 1);
        cipher_block_of_pages<2, ROUNDS>(job, lane);
        r = r2;
      }
    }
    for (; p < c1; ++p) {
      while (reqs[r].page_end <= p) ++r;
      PageJob job[1];
      job_from_request(job[0], reqs + r, keys, p);
      cipher_block_of_pages<1, ROUNDS>(job, lane);
    }
  }
}

// --------------------------------------------------------------- probes ---

// Streaming copy: the HBM reference point for the page kernels (same
// dwordx4 accesses, no arithmetic).
__global__ __launch_bounds__(kBlockThreads) void copy_probe_kernel(
    const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlockThreads;
  uint64_t i = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i];
    const uint4 b = src[i + stride];
    const uint4 c = src[i + 2 * stride];
    const uint4 e = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = e;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
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

template <int ROUNDS>
hipError_t launch_plain_r(const PlainArgs& a, uint32_t kind,
                          hipStream_t stream) {
  const uint64_t blocks = (a.n_pages + kWavesPerBlock - 1) / kWavesPerBlock;
  if (kind == kNonceArray)
    hipLaunchKernelGGL((plain_pages_kernel<ROUNDS, kNonceArray>),
                       dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream,
                       a);
  else
    hipLaunchKernelGGL((plain_pages_kernel<ROUNDS, kNonceLinear>),
                       dim3((uint32_t)blocks), dim3(kBlockThreads), 0, stream,
                       a);
  return hipGetLastError();
}

}  // namespace

// A plain launch covers at most this many pages; longer runs are split so
// that the grid stays far below the 2^32 work-item limit of one dispatch.
constexpr uint64_t kMaxPagesPerPlainLaunch = 1ull << 24;

hipError_t launch_plain(const PlainArgs& a, uint32_t kind, int rounds,
                        hipStream_t stream) {
  for (uint64_t done = 0; done < a.n_pages;) {
    PlainArgs part = a;
    part.first_page = a.first_page + done;
    part.n_pages = a.n_pages - done;
    if (part.n_pages > kMaxPagesPerPlainLaunch)
      part.n_pages = kMaxPagesPerPlainLaunch;
    hipError_t e;
    switch (rounds) {
      case 20: e = launch_plain_r<20>(part, kind, stream); break;
      case 12: e = launch_plain_r<12>(part, kind, stream); break;
      case 8: e = launch_plain_r<8>(part, kind, stream); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    done += part.n_pages;
  }
  return hipSuccess;
}

const void* batch_kernel_fn(uint32_t unroll, int rounds) {
  if (unroll == 2) {
    switch (rounds) {
      case 20: return reinterpret_cast<const void*>(&batch_pages_kernel<20, 2>);
      case 12: return reinterpret_cast<const void*>(&batch_pages_kernel<12, 2>);
      case 8: return reinterpret_cast<const void*>(&batch_pages_kernel<8, 2>);
    }
  } else if (unroll == 1) {
    switch (rounds) {
      case 20: return reinterpret_cast<const void*>(&batch_pages_kernel<20, 1>);
      case 12: return reinterpret_cast<const void*>(&batch_pages_kernel<12, 1>);
      case 8: return reinterpret_cast<const void*>(&batch_pages_kernel<8, 1>);
    }
  }
  return nullptr;
}

hipError_t launch_batch(const DevBatchHdr* batch, const uint32_t* keys,
                        uint32_t pages_per_wave, uint32_t unroll,
                        uint32_t grid_blocks, int rounds, hipStream_t stream) {
  const void* fn = batch_kernel_fn(unroll, rounds);
  if (!fn || pages_per_wave == 0 || grid_blocks == 0)
    return hipErrorInvalidValue;
  void* args[] = {(void*)&batch, (void*)&keys, (void*)&pages_per_wave};
  return hipLaunchKernel(fn, dim3(grid_blocks), dim3(kBlockThreads), args, 0,
                         stream);
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes,
                       uint32_t grid_blocks, hipStream_t stream) {
  if (bytes % 16 != 0 || grid_blocks == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_probe_kernel, dim3(grid_blocks),
                     dim3(kBlockThreads), 0, stream,
                     reinterpret_cast<const uint4*>(src),
                     reinterpret_cast<uint4*>(dst), bytes / 16);
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
