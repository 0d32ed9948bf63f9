// Device building blocks of the ChaCha page cipher for gfx950, shared by the
// launch-per-call kernels (page_cipher.hip) and the resident-key kernel
// (resident.hip).  What they compute and how it maps to the hardware is
// described at the top of page_cipher.hip.
#pragma once

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

// ------------------------------------------------------------- Salsa20 ---
// The second cipher behind the same page interface: Salsa20 (Bernstein,
// 2008), ChaCha's predecessor.  Its state is
//   [ c0 k0 k1 k2 | k3 c1 v0 v1 | t0 t1 c2 k4 | k5 k6 k7 c3 ]
// with the sigma words c, the key words k, the 64-bit nonce v (page nonce
// words 0, 1) and the 64-bit block counter t: t0 = the block index j (the
// lane), t1 = page nonce word 2.  Its quarter round on (a, b, c, d) updates
// b, c, d, a by xor with a rotated sum; a double round is a column round on
// (0,4,8,12) (5,9,13,1) (10,14,2,6) (15,3,7,11) and a row round on
// (0,1,2,3) (5,6,7,4) (10,11,8,9) (15,12,13,14).

// Salsa20 quarter round on wave-uniform words (scalar unit).
__device__ __forceinline__ void salsa_quarter_s(uint32_t& a, uint32_t& b,
                                                uint32_t& c, uint32_t& d) {
  b ^= srotl32<7>(a + d);
  c ^= srotl32<9>(b + a);
  d ^= srotl32<13>(c + b);
  a ^= srotl32<18>(d + c);
}

#define MS_SALSA_QUARTER(a, b, c, d)                                  \
  b ^= rotl32(a + d, 7); c ^= rotl32(b + a, 9); d ^= rotl32(c + b, 13); \
  a ^= rotl32(d + c, 18);

// Salsa20 keystream block `ctr` (the lane id), feed-forward included.  Only
// word 8 depends on the lane at the start, so the first double round runs
// five of its eight quarter rounds, and the uniform steps of the other
// three, on the scalar unit.
template <int ROUNDS>
__device__ __forceinline__ void salsa_keystream(uint32_t (&o)[16],
                                                const uint32_t (&key)[8],
                                                const uint32_t (&nonce)[3],
                                                uint32_t ctr) {
  uint32_t k[8], n[3];
#pragma unroll
  for (int i = 0; i < 8; ++i) k[i] = uni(key[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i) n[i] = uni(nonce[i]);
  uint32_t x0 = kSigma0, x1 = k[0], x2 = k[1], x3 = k[2], x4 = k[3],
           x5 = kSigma1, x6 = n[0], x7 = n[1], x8, x9 = n[2], x10 = kSigma2,
           x11 = k[4], x12 = k[5], x13 = k[6], x14 = k[7], x15 = kSigma3;
  // first column round: (0,4,8,12) meets the counter at its second step
  x4 ^= srotl32<7>(x0 + x12);
  x8 = ctr ^ srotl32<9>(x4 + x0);
  x12 ^= rotl32(x8 + x4, 13);
  x0 ^= rotl32(x12 + x8, 18);
  salsa_quarter_s(x5, x9, x13, x1);
  salsa_quarter_s(x10, x14, x2, x6);
  salsa_quarter_s(x15, x3, x7, x11);
  // first row round: (5,6,7,4) is still uniform; (10,11,8,9) and
  // (15,12,13,14) start with uniform steps
  MS_SALSA_QUARTER(x0, x1, x2, x3);
  salsa_quarter_s(x5, x6, x7, x4);
  x11 ^= srotl32<7>(x10 + x9);
  x8 ^= srotl32<9>(x11 + x10);
  x9 ^= rotl32(x8 + x11, 13);
  x10 ^= rotl32(x9 + x8, 18);
  x12 ^= srotl32<7>(x15 + x14);
  x13 ^= rotl32(x12 + x15, 9);
  x14 ^= rotl32(x13 + x12, 13);
  x15 ^= rotl32(x14 + x13, 18);
#pragma unroll
  for (int r = 2; r < ROUNDS; r += 2) {
    MS_SALSA_QUARTER(x0, x4, x8, x12);
    MS_SALSA_QUARTER(x5, x9, x13, x1);
    MS_SALSA_QUARTER(x10, x14, x2, x6);
    MS_SALSA_QUARTER(x15, x3, x7, x11);
    MS_SALSA_QUARTER(x0, x1, x2, x3);
    MS_SALSA_QUARTER(x5, x6, x7, x4);
    MS_SALSA_QUARTER(x10, x11, x8, x9);
    MS_SALSA_QUARTER(x15, x12, x13, x14);
  }
  o[0] = x0 + kSigma0; o[1] = x1 + k[0]; o[2] = x2 + k[1]; o[3] = x3 + k[2];
  o[4] = x4 + k[3]; o[5] = x5 + kSigma1; o[6] = x6 + n[0]; o[7] = x7 + n[1];
  o[8] = x8 + ctr; o[9] = x9 + n[2]; o[10] = x10 + kSigma2;
  o[11] = x11 + k[4]; o[12] = x12 + k[5]; o[13] = x13 + k[6];
  o[14] = x14 + k[7]; o[15] = x15 + kSigma3;
}

// Keystream of the selected cipher.
template <uint32_t CIPHER, int ROUNDS>
__device__ __forceinline__ void cipher_keystream(uint32_t (&o)[16],
                                                 const uint32_t (&key)[8],
                                                 const uint32_t (&nonce)[3],
                                                 uint32_t ctr) {
  if constexpr (CIPHER == kCipherSalsa)
    salsa_keystream<ROUNDS>(o, key, nonce, ctr);
  else
    keystream<ROUNDS>(o, key, nonce, ctr);
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
template <int ROUNDS, uint32_t CIPHER = kCipherChaCha>
__device__ __forceinline__ void cipher_page(uint4 (&v)[4], const PageJob& j,
                                            const uint32_t (&k)[8],
                                            uint4* lds, uint32_t lane) {
  uint32_t o[16];
  cipher_keystream<CIPHER, ROUNDS>(o, k, j.n, lane);
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
template <int ROUNDS, int UNROLL, uint32_t CIPHER = kCipherChaCha,
          class PageSource>
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
      cipher_page<ROUNDS, CIPHER>(a, ja, k, lds, lane);
      if (!more_b) break;
      const bool more_a = pages.next(ja);
      if (more_a) load_page(a, ja, lane);
      pages.key(jb, k);
      cipher_page<ROUNDS, CIPHER>(b, jb, k, lds, lane);
      if (!more_a) break;
    }
  } else {
    do {
      load_page(a, ja, lane);
      pages.key(ja, k);
      cipher_page<ROUNDS, CIPHER>(a, ja, k, lds, lane);
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

}  // namespace
}  // namespace ms
