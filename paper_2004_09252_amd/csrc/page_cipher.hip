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
// The plain kernel takes one run of pages with one key and one nonce rule.
// The batched kernel walks a flattened list of (request, page) items, each
// request with its own key slot and nonce rule, taking `pages_per_wave`
// consecutive items at a time.
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

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t rotl32(uint32_t v, uint32_t n) {
  return (v << n) | (v >> (32u - n));
}

// Values that are wave-uniform by construction but that the compiler may
// have loaded into vector registers (e.g. descriptor fields read after the
// kernel has stored to global memory) are pinned to scalar registers here.
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Read-only tables (key table, request descriptors, nonce arrays) are read
// through the constant address space: the compiler may then use scalar loads
// for them anywhere in a kernel, also after the kernel's own global stores.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cnst(
    const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Rotate of a wave-uniform value on the scalar unit (there is no scalar
// rotate instruction; left shift, right shift and or).
template <int N>
__device__ __forceinline__ uint32_t srotl32(uint32_t v) {
  uint32_t r, t;
  asm("s_lshl_b32 %0, %2, %3\n\ts_lshr_b32 %1, %2, %4\n\ts_or_b32 %0, %0, %1"
      : "=&s"(r), "=&s"(t)
      : "s"(v), "i"(N), "i"(32 - N)
      : "scc");
  return r;
}

// Quarter round on wave-uniform words (scalar unit).
__device__ __forceinline__ void quarter_s(uint32_t& a, uint32_t& b, uint32_t& c,
                                          uint32_t& d) {
  a += b; d = srotl32<16>(d ^ a);
  c += d; b = srotl32<12>(b ^ c);
  a += b; d = srotl32<8>(d ^ a);
  c += d; b = srotl32<7>(b ^ c);
}

#define MS_QUARTER(a, b, c, d)                          \
  a += b; d = rotl32(d ^ a, 16); c += d; b = rotl32(b ^ c, 12); \
  a += b; d = rotl32(d ^ a, 8);  c += d; b = rotl32(b ^ c, 7);

// Wave-uniform description of one page: where it is, its nonce, and (for
// batches) the key-table row of its request.
struct PageJob {
  const uint4* src;
  uint4* dst;
  uint32_t n[3];
  uint32_t slot;
};

// Keystream block `ctr` (the lane id) for key k and nonce n, feed-forward
// included.  The first double round is split into its uniform (scalar) and
// lane-dependent (vector) parts; the rest is the plain round function.
template <int ROUNDS>
__device__ __forceinline__ void keystream(uint32_t (&o)[16],
                                          const uint32_t (&key)[8],
                                          const uint32_t (&nonce)[3],
                                          uint32_t ctr) {
  uint32_t k[8], n[3];
#pragma unroll
  for (int i = 0; i < 8; ++i) k[i] = uni(key[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) n[i] = uni(nonce[i]);
  uint32_t x0, x1, x2, x3, x4, x5, x6, x7, x8, x9, x10, x11, x12, x13, x14,
      x15;
  // first column round: columns 1..3 hold no counter word
  x1 = kSigma1; x5 = k[1]; x9 = k[5]; x13 = n[0];
  quarter_s(x1, x5, x9, x13);
  x2 = kSigma2; x6 = k[2]; x10 = k[6]; x14 = n[1];
  quarter_s(x2, x6, x10, x14);
  x3 = kSigma3; x7 = k[3]; x11 = k[7]; x15 = n[2];
  quarter_s(x3, x7, x11, x15);
  // column 0 meets the counter after its first add
  {
    const uint32_t a0 = kSigma0 + k[0];
    x12 = rotl32(ctr ^ a0, 16);
    x8 = k[4] + x12;
    x4 = rotl32(k[0] ^ x8, 12);
    x0 = a0 + x4;
    x12 = rotl32(x12 ^ x0, 8);
    x8 += x12;
    x4 = rotl32(x4 ^ x8, 7);
  }
  // first diagonal round: (1,6,11,12) starts with a uniform add and
  // (2,7,8,13) with a uniform add, xor and rotate
  MS_QUARTER(x0, x5, x10, x15);
  x1 += x6;
  x12 = rotl32(x12 ^ x1, 16); x11 += x12; x6 = rotl32(x6 ^ x11, 12);
  x1 += x6; x12 = rotl32(x12 ^ x1, 8); x11 += x12; x6 = rotl32(x6 ^ x11, 7);
  x2 += x7; x13 = srotl32<16>(x13 ^ x2);
  x8 += x13; x7 = rotl32(x7 ^ x8, 12);
  x2 += x7; x13 = rotl32(x13 ^ x2, 8); x8 += x13; x7 = rotl32(x7 ^ x8, 7);
  MS_QUARTER(x3, x4, x9, x14);
#pragma unroll
  for (int r = 2; r < ROUNDS; r += 2) {
    MS_QUARTER(x0, x4, x8, x12);
    MS_QUARTER(x1, x5, x9, x13);
    MS_QUARTER(x2, x6, x10, x14);
    MS_QUARTER(x3, x7, x11, x15);
    MS_QUARTER(x0, x5, x10, x15);
    MS_QUARTER(x1, x6, x11, x12);
    MS_QUARTER(x2, x7, x8, x13);
    MS_QUARTER(x3, x4, x9, x14);
  }
  o[0] = x0 + kSigma0; o[1] = x1 + kSigma1;
  o[2] = x2 + kSigma2; o[3] = x3 + kSigma3;
  o[4] = x4 + k[0]; o[5] = x5 + k[1]; o[6] = x6 + k[2]; o[7] = x7 + k[3];
  o[8] = x8 + k[4]; o[9] = x9 + k[5]; o[10] = x10 + k[6]; o[11] = x11 + k[7];
  o[12] = x12 + ctr; o[13] = x13 + n[0]; o[14] = x14 + n[1];
  o[15] = x15 + n[2];
}

// Page data always lives in global memory; saying so lets the compiler use
// global (not flat) loads and stores also where the pointers come from
// descriptors.
typedef __attribute__((address_space(1))) v4u gv4u;

__device__ __forceinline__ uint4 load_nt(const uint4* p) {
  const v4u v = __builtin_nontemporal_load((const gv4u*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_nt(uint4 a, uint4* p) {
  const v4u v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, (gv4u*)p);
}

// 16-byte slot i (0..255) of the per-wave keystream buffer, XOR-swizzled so
// that both the block-order writes (i = 4*lane + q) and the consecutive-order
// reads (i = 64*q + lane) spread over all LDS banks.
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) {
  return i ^ ((i >> 3) & 7u);
}

// A wave's LDS accesses to its own buffer must not be reordered across this
// point (the hardware keeps one wave's LDS operations in order).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coalesced load of a whole page: access q of lane l is 16-byte column
// 64*q + l.
__device__ __forceinline__ void load_page(uint4 (&v)[4], const PageJob& j,
                                          uint32_t lane) {
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = load_nt(j.src + q * 64 + lane);
}

// Keystream for the page, transposed through LDS, XORed over the loaded
// data and stored coalesced.
template <int ROUNDS>
__device__ __forceinline__ void cipher_page(uint4 (&v)[4], const PageJob& j,
                                            const uint32_t (&k)[8],
                                            uint4* lds, uint32_t lane) {
  uint32_t o[16];
  keystream<ROUNDS>(o, k, j.n, lane);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    lds[lds_slot(lane * 4 + q)] =
        make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  wave_lds_order();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 ks = lds[lds_slot(q * 64 + lane)];
    uint4 r = v[q];
    r.x ^= ks.x;
    r.y ^= ks.y;
    r.z ^= ks.z;
    r.w ^= ks.w;
    store_nt(r, j.dst + q * 64 + lane);
  }
  wave_lds_order();
}

// Walk the pages a PageSource hands out.  UNROLL 2 keeps the next page's
// loads in flight while the current page is ciphered (two register buffers,
// no copies); UNROLL 1 loads, ciphers and stores one page at a time.  The
// source also supplies each page's key (fixed for plain launches, looked up
// in the key table per request for batches).
template <int ROUNDS, int UNROLL, class PageSource>
__device__ __forceinline__ void run_pages(PageSource& pages, uint4* lds,
                                          uint32_t lane) {
  PageJob ja, jb;
  if (!pages.next(ja)) return;
  uint4 a[4], b[4];
  uint32_t k[8];
  if (UNROLL == 2) {
    load_page(a, ja, lane);
    for (;;) {
      const bool more_b = pages.next(jb);
      if (more_b) load_page(b, jb, lane);
      pages.key(ja, k);
      cipher_page<ROUNDS>(a, ja, k, lds, lane);
      if (!more_b) break;
      const bool more_a = pages.next(ja);
      if (more_a) load_page(a, ja, lane);
      pages.key(jb, k);
      cipher_page<ROUNDS>(b, jb, k, lds, lane);
      if (!more_a) break;
    }
  } else {
    do {
      load_page(a, ja, lane);
      pages.key(ja, k);
      cipher_page<ROUNDS>(a, ja, k, lds, lane);
    } while (pages.next(ja));
  }
}

__device__ __forceinline__ uint32_t wave_in_block() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ void load_key(uint32_t (&k)[8], const uint32_t* keys,
                                         uint32_t slot) {
  const uint32_t* p = keys + (uint64_t)slot * 8u;
#pragma unroll
  for (int i = 0; i < 8; ++i) k[i] = p[i];
}

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

template <int ROUNDS, int UNROLL, uint32_t KIND>
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
  run_pages<ROUNDS, UNROLL>(src, lds[w], lane);
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

template <int ROUNDS, int UNROLL>
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
  run_pages<ROUNDS, UNROLL>(s, lds, lane);
}

// Descriptors in device memory (copied there before the launch).
template <int ROUNDS, int UNROLL>
__global__ __launch_bounds__(kBlockThreads, UNROLL == 2 ? 7 : 8) void batch_pages_kernel(
    const DevBatchHdr* __restrict__ hdr, const uint32_t* __restrict__ keys,
    uint32_t pages_per_wave) {
  __shared__ uint4 lds[kWavesPerBlock][256];
  const uint32_t w = wave_in_block();
  batch_body<ROUNDS, UNROLL>(hdr, reinterpret_cast<const DevReq*>(hdr + 1),
                             keys, pages_per_wave, lds[w], w);
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

template <int ROUNDS, int UNROLL>
hipError_t launch_plain_ru(const PlainArgs& a, uint32_t kind, uint32_t grid,
                           hipStream_t stream) {
  if (kind == kNonceArray)
    hipLaunchKernelGGL((plain_pages_kernel<ROUNDS, UNROLL, kNonceArray>),
                       dim3(grid), dim3(kBlockThreads), 0, stream, a);
  else
    hipLaunchKernelGGL((plain_pages_kernel<ROUNDS, UNROLL, kNonceLinear>),
                       dim3(grid), dim3(kBlockThreads), 0, stream, a);
  return hipGetLastError();
}

template <int ROUNDS>
hipError_t launch_plain_r(const PlainArgs& a, uint32_t kind, uint32_t grid,
                          uint32_t unroll, hipStream_t stream) {
  return unroll == 2 ? launch_plain_ru<ROUNDS, 2>(a, kind, grid, stream)
                     : launch_plain_ru<ROUNDS, 1>(a, kind, grid, stream);
}

}  // namespace

// A plain launch covers at most this many pages (32-bit page counters in the
// kernel); longer runs are split into several launches.
constexpr uint64_t kMaxPagesPerPlainLaunch = 1ull << 24;

hipError_t launch_plain(const PlainArgs& a, uint32_t kind, int rounds,
                        uint32_t max_waves, uint32_t unroll,
                        hipStream_t stream) {
  if (max_waves == 0 || (unroll != 1 && unroll != 2))
    return hipErrorInvalidValue;
  if (rounds != 20 && rounds != 12 && rounds != 8) return hipErrorInvalidValue;
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
    hipError_t e = hipErrorInvalidValue;
    switch (rounds) {
      case 20: e = launch_plain_r<20>(part, kind, grid, unroll, stream); break;
      case 12: e = launch_plain_r<12>(part, kind, grid, unroll, stream); break;
      case 8: e = launch_plain_r<8>(part, kind, grid, unroll, stream); break;
    }
    if (e != hipSuccess) return e;
    done += part.n_pages;
  }
  return hipSuccess;
}

const void* plain_kernel_fn(uint32_t unroll, int rounds, uint32_t kind) {
#define MS_PLAIN_FN(R, U)                                                   \
  (kind == kNonceArray                                                      \
       ? reinterpret_cast<const void*>(&plain_pages_kernel<R, U, kNonceArray>) \
       : reinterpret_cast<const void*>(&plain_pages_kernel<R, U, kNonceLinear>))
  if (unroll == 2) {
    switch (rounds) {
      case 20: return MS_PLAIN_FN(20, 2);
      case 12: return MS_PLAIN_FN(12, 2);
      case 8: return MS_PLAIN_FN(8, 2);
    }
  } else if (unroll == 1) {
    switch (rounds) {
      case 20: return MS_PLAIN_FN(20, 1);
      case 12: return MS_PLAIN_FN(12, 1);
      case 8: return MS_PLAIN_FN(8, 1);
    }
  }
#undef MS_PLAIN_FN
  return nullptr;
}

uint32_t resident_waves_per_cu(const void* fn) {
  int blocks = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &blocks, fn, kBlockThreads, 0) != hipSuccess ||
      blocks <= 0)
    return 0;
  return (uint32_t)blocks * kWavesPerBlock;
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
