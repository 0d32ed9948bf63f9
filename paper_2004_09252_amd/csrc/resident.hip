// Resident-key page cipher for gfx950: MemShield's own GPU design (section
// 4.4) on CDNA4.
//
// The paper keeps its 256-bit key only in the registers of a GPU kernel that
// never ends, and feeds that kernel pages through a multiple-producer ring
// in memory mapped between host and device; host threads enqueue pages, GPU
// workers take them.  Here:
//   * one dispatch, on an HSA queue of its own (so no stream of the HIP
//     runtime can wait behind it), holds `n_workers` worker waves plus one
//     poller wave for as long as the host keeps it;
//   * the key reaches the kernel once, through a 32-byte device buffer: each
//     worker reads it with cache-bypassing vector loads into SGPRs (the
//     compiler may not move it elsewhere: it is opaque after an empty asm),
//     counts itself in, and the last worker zeroes the buffer and tells the
//     host; from then on the key exists only in registers (no scratch: the
//     kernel's resource usage is checked to be spill-free);
//   * an engine that serves a context's own requests (its serving stage)
//     holds no key of its own: a descriptor names a row of the context's
//     device key table, which the worker reads with system-scope loads for
//     each descriptor (the key then lives in HBM, as for the launch-per-call
//     kernels, and a row may be reloaded between descriptors);
//   * an engine may instead hold up to kRkMaxKeys keys (one per client, say):
//     each workgroup copies them into a table in its LDS before its waves
//     start, the last worker wipes the device buffer as above, and a worker
//     moves the key its descriptor names from LDS into SGPRs; the keys then
//     live only on chip (LDS and registers), never in HBM or host memory;
//   * the host writes 64-byte descriptors (a run of pages in pinned host
//     memory or in device memory, its linear nonce, its key index) into a
//     ring in pinned host memory and publishes a count; the
//     poller wave reads that count over the link and mirrors it into device
//     memory, so the idle workers wait on device memory instead of polling
//     across the link;
//   * each worker owns a fixed share of the ring positions, every W-th (W
//     workers), so taking work needs no atomic; the shares are strided so
//     that position q belongs to worker (q mod W) * s mod W, with s >= 4
//     coprime to W: the pages of one request land in different workgroups,
//     hence on different compute units and XCDs;
//   * a worker reads its descriptor and the pages with system-scope loads
//     (coalesced 8-byte columns, no stale cached copy is possible, whether a
//     page is in host memory or in HBM), XORs the
//     keystream, transposed through LDS as in the launch-per-call kernels,
//     writes the pages back with system-scope stores, and once those stores
//     are acknowledged writes the position into the slot's completion word,
//     which the host polls;
//   * every wait is bounded: the poller leaves when the host sets `stop` or
//     after `idle_ticks` without host activity, and the workers leave when
//     the poller does, so the launch always drains;
//   * control flow is wave-uniform everywhere (no lane-masked branches): a
//     value one lane obtains (the key-load count) comes from an atomic all
//     lanes execute, lane 0 adding 1 and the others 0, and control words are
//     stored by all lanes with the same value.  A lane-0-only branch next to
//     a loop back-edge can otherwise be compiled into an exec-mask loop that
//     some lanes leave and others do not.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cipher_core.h"
#include "ms_resident_kernel.h"

namespace ms {
namespace {

__device__ __forceinline__ uint64_t ld_sys64(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_sys32(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Page data: global address space (the addresses arrive as integers in the
// descriptors), system scope.
typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ __forceinline__ uint64_t ld_page(uint64_t addr) {
  return __hip_atomic_load(reinterpret_cast<gu64*>(addr), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_page(uint64_t addr, uint64_t v) {
  __hip_atomic_store(reinterpret_cast<gu64*>(addr), v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_dev64(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev32(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The poller: mirror the host's published count into device memory; leave
// on `stop` or after idle_ticks without a new descriptor or heartbeat.
__device__ void poll_host(const RkArgs& a, uint32_t lane) {
  uint64_t last_pub = 0, last_hb = 0;
  uint64_t t_last = wall_clock64();
  for (;;) {
    // the three control words in one round trip over the link
    const uint32_t stop = ld_sys32(&a.hctl->stop);
    const uint64_t pub = uni64(ld_sys64(&a.hctl->published));
    const uint64_t hb = uni64(ld_sys64(&a.hctl->heartbeat));
    if (uni(stop)) break;
    const uint64_t now = wall_clock64();
    if (pub != last_pub) {
      // A relaxed store: the count orders nothing this wave wrote.  The
      // descriptors it covers were written by the host before the host's
      // count, and a worker reads them with system-scope loads only after it
      // sees this count, so they reach it whole.  (A release here would
      // write back the L2 at every new count.)
      __hip_atomic_store(&a.dctl->published, pub, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      last_pub = pub;
      t_last = now;
    } else if (hb != last_hb) {
      last_hb = hb;
      t_last = now;
    } else if (a.idle_ticks != 0 && now - t_last > a.idle_ticks) {
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(&a.dctl->stop, 1u, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&a.hctl->exited, 1u, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// Cipher n_pages consecutive pages from `src` to `dst` (GPU-visible
// addresses) with the key whose words are `kv` (the same in every lane, not
// yet made wave-uniform).  ARRAY: page p's nonce is the 12 bytes at nb +
// 12p (every lane reads them); otherwise it is LE64(nb + p*ns) || tag.
template <uint32_t CIPHER, int ROUNDS, bool ARRAY>
__device__ __forceinline__ void cipher_run(const uint32_t (&kv)[8],
                                           uint64_t src, uint64_t dst,
                                           uint64_t nb, uint64_t ns,
                                           uint32_t tag, uint32_t n_pages,
                                           uint4* lds, uint32_t lane) {
  uint32_t kk[8];  // the key in SGPRs, filled below
  // the page's 512 8-byte units: access q of lane l is unit 64*q + l
  auto load = [&](uint64_t (&v)[8], uint32_t p) {
    const uint64_t s = src + (uint64_t)p * kPageBytes;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = ld_page(s + 8u * (q * 64 + lane));
  };
  auto cipher = [&](const uint64_t (&v)[8], uint32_t p) {
    const uint64_t o = dst + (uint64_t)p * kPageBytes;
    uint32_t n[3];
    if (ARRAY) {
      const uint32_t* na =
          reinterpret_cast<const uint32_t*>(nb + (uint64_t)p * 12u);
      n[0] = uni(ld_sys32(na));
      n[1] = uni(ld_sys32(na + 1));
      n[2] = uni(ld_sys32(na + 2));
    } else {
      const uint64_t nv = nb + (uint64_t)p * ns;
      n[0] = (uint32_t)nv;
      n[1] = (uint32_t)(nv >> 32);
      n[2] = tag;
    }
    uint32_t ks[16];
    // block `lane` = bytes 64*lane..
    cipher_keystream<CIPHER, ROUNDS>(ks, kk, n, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      lds[lds_slot(lane * 4 + q)] =
          make_uint4(ks[4 * q], ks[4 * q + 1], ks[4 * q + 2], ks[4 * q + 3]);
    wave_lds_order();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t unit = q * 64 + lane;  // bytes 8*unit .. 8*unit+7
      const uint2 x = reinterpret_cast<const uint2*>(
          &lds[lds_slot(unit >> 1)])[unit & 1];
      st_page(o + 8u * unit, v[q] ^ (((uint64_t)x.y << 32) | x.x));
    }
    wave_lds_order();
  };
  // Two page buffers: the next page's loads are in flight while the
  // current page's keystream is computed and stored (a worker is the only
  // wave on its SIMD, so nothing else would hide that latency).  The page
  // count is wave-uniform, so these branches are scalar.
  uint64_t va[8], vb[8];
  load(va, 0);
  // The key words become wave-uniform only now: waiting for them here lets
  // their load (for the serving ring, a system-scope read of the key table)
  // overlap the first page's loads instead of preceding them.  The asm
  // keeps each word in an SGPR, opaque to the compiler.
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    kk[i] = uni(kv[i]);
    asm volatile("" : "+s"(kk[i]) : : "memory");
  }
  for (uint32_t p = 0;; p += 2) {
    const bool more_b = p + 1 < n_pages;
    if (more_b) load(vb, p + 1);
    cipher(va, p);
    if (!more_b) break;
    const bool more_a = p + 2 < n_pages;
    if (more_a) load(va, p + 2);
    cipher(vb, p + 1);
    if (!more_a) break;
  }
}

// Cipher the pages of the descriptor at ring position `pos`, then mark the
// position complete.  A descriptor that does not carry its own position, has
// a page count outside 1..max_pages, a key index outside the engine's keys
// or an unknown nonce kind is not touched and raises `error`.  `k` is the
// key of a one-key engine; `keytab` the LDS key table of a many-key engine.
template <uint32_t CIPHER, int ROUNDS>
__device__ void serve_one(const RkArgs& a, const uint32_t (&k)[8],
                          const uint32_t* keytab, uint64_t pos, uint4* lds,
                          uint32_t lane) {
  // the descriptor in one 64-byte read: lane l loads its word l % 8 (the
  // lanes past 7 repeat those addresses, which the wave's load merges), and
  // each field is taken from the lane that holds it
  const uint64_t wv = ld_sys64(reinterpret_cast<const uint64_t*>(
                                   a.ring + (pos & a.ring_mask)) +
                               (lane & 7u));
  const uint32_t wlo = (uint32_t)wv, whi = (uint32_t)(wv >> 32);
  auto field = [&](int i) -> uint64_t {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)whi, i) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)wlo, i);
  };
  static_assert(offsetof(RkDesc, seq) == 32 && offsetof(RkDesc, n_pages) == 40 &&
                    offsetof(RkDesc, key) == 48,
                "descriptor words");
  const uint64_t src = field(0);
  const uint64_t dst = field(1);
  const uint64_t nb = field(2);
  const uint64_t ns = field(3);
  const uint64_t seq = field(4);
  const uint64_t pt = field(5);  // n_pages | tag << 32
  const uint64_t kk64 = field(6);  // key | kind << 32
  const uint32_t key = (uint32_t)kk64;
  const uint32_t kind = (uint32_t)(kk64 >> 32);
  const uint32_t n_pages = (uint32_t)pt;
  const uint32_t tag = (uint32_t)(pt >> 32);
  const uint32_t key_limit = a.n_keys ? a.n_keys : a.table_rows;
  if (seq != pos || n_pages == 0 || n_pages > a.max_pages ||
      key >= key_limit || kind > 1) {
    st_sys32(&a.hctl->error, 1u);
  } else {
    // the key's words (cipher_run makes them uniform once the first
    // page's loads are issued)
    uint32_t kv[8];
    if (a.n_keys == 0) {
      // a row of the context's key table, fresh for every descriptor
#pragma unroll
      for (int i = 0; i < 8; ++i)
        kv[i] = ld_sys32(a.key_table + (uint64_t)key * 8u + i);
    } else if (a.n_keys > 1) {
#pragma unroll
      for (int i = 0; i < 8; ++i) kv[i] = keytab[key * 8u + i];
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) kv[i] = k[i];
    }
    // the nonce kind is decided once per descriptor, outside the page loop
    if (kind == 0)
      cipher_run<CIPHER, ROUNDS, true>(kv, src, dst, nb, ns, tag, n_pages,
                                       lds, lane);
    else
      cipher_run<CIPHER, ROUNDS, false>(kv, src, dst, nb, ns, tag, n_pages,
                                        lds, lane);
  }
  // The page stores are complete before the completion word is written.
  // Every global store of this worker since its last completion word is a
  // system-scope store, which the L2 writes through instead of holding
  // dirty, so waiting for those stores to be acknowledged orders them before
  // the completion store (the asm's memory clobber keeps the compiler from
  // moving either across it).  A release fence would add a write-back of
  // the whole L2, which serializes across the device: with one descriptor
  // per page, a 256-page request took 33 us that way against 13 us so.
  asm volatile("s_waitcnt vmcnt(0)" : : : "memory");
  st_sys64(&a.completed[pos & a.ring_mask], pos + 1);
}

template <uint32_t CIPHER, int ROUNDS>
__device__ void serve_ring(const RkArgs& a, const uint32_t* keytab,
                           uint4* lds, uint32_t lane, uint32_t worker) {
  uint32_t k[8];
  if (a.n_keys == 1) {  // (0: key-table rows; 2..: the LDS table)
#pragma unroll
    for (int i = 0; i < 8; ++i) k[i] = uni(ld_sys32(a.key_buf + i));
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) k[i] = 0;  // keys come from `keytab`
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) asm volatile("" : "+s"(k[i]) : : "memory");
  // one count per wave: lane 0 adds 1, the other lanes 0; lane 0's result
  // is the count before this wave
  const uint32_t before = uni(__hip_atomic_fetch_add(
      &a.dctl->key_loads, lane == 0 ? 1u : 0u, __ATOMIC_ACQ_REL,
      __HIP_MEMORY_SCOPE_AGENT));
  if (before + 1 == a.n_workers) {
    // every worker now holds the keys (registers, or its workgroup's LDS
    // table): wipe the memory copy; lanes past the end repeat the last word
    const uint32_t words = a.n_keys * 8u;
    for (uint32_t i = 0; i < words; i += kWave)
      st_sys32(a.key_buf + min(i + lane, words - 1), 0u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    st_sys32(&a.hctl->ready, 1u);
  }
  // this worker's share of the ring: the positions congruent to
  // worker * inv_step (the inverse of the stride) modulo n_workers
  // (the product is below n_workers squared, which fits 32 bits, and a
  // 32-bit division compiles to straight-line code)
  const uint32_t first = uni((worker * a.inv_step) % a.n_workers);
  for (uint64_t pos = first;; pos += a.n_workers) {
    if (uni(ld_dev32(&a.dctl->stop))) return;
    // wait on device memory until the position is published, or stop; the
    // worker holding the next position to be published polls fastest, the
    // next 63 (the rest of a request of up to 64 descriptors) every ~500
    // cycles, the others every ~4000, which keeps the load on the word low
    for (;;) {
      const uint64_t pub = uni64(ld_dev64(&a.dctl->published));
      if (pos < pub) break;
      if (uni(ld_dev32(&a.dctl->stop))) return;
      if (pos == pub)
        __builtin_amdgcn_s_sleep(2);
      else if (pos - pub < 64)
        __builtin_amdgcn_s_sleep(8);
      else
        __builtin_amdgcn_s_sleep(64);
    }
    serve_one<CIPHER, ROUNDS>(a, k, keytab, pos, lds, lane);
  }
}

template <uint32_t CIPHER, int ROUNDS>
__device__ __forceinline__ void resident_pages(const RkArgs& a) {
  __shared__ uint4 lds[kWavesPerBlock][256];
  __shared__ uint32_t keytab[kRkMaxKeys * 8];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t w = wave_in_block();
  const uint32_t gw = blockIdx.x * kWavesPerBlock + w;
  if (a.n_keys > 1) {
    // many keys: the whole workgroup copies the table into LDS; threads past
    // the end repeat the last word
    const uint32_t words = a.n_keys * 8u;
    for (uint32_t i = 0; i < words; i += kBlockThreads) {
      const uint32_t j = min(i + threadIdx.x, words - 1);
      keytab[j] = ld_sys32(a.key_buf + j);
    }
  }
  __syncthreads();
  if (gw == 0) {
    poll_host(a, lane);
    return;
  }
  if (gw > a.n_workers) return;
  serve_ring<CIPHER, ROUNDS>(a, keytab, lds[w], lane, gw - 1);
}

}  // namespace
}  // namespace ms

// Entry points by cipher and round count (r: ChaCha, s: Salsa20).  This
// file is built as its own code object and dispatched by resident.cpp on a
// private HSA queue, so the names are plain C symbols.
#define MS_RESIDENT_ENTRY(NAME, CIPHER, ROUNDS)                       \
  extern "C" __global__ __launch_bounds__(ms::kBlockThreads) void NAME( \
      ms::RkArgs a) {                                                  \
    ms::resident_pages<CIPHER, ROUNDS>(a);                             \
  }
MS_RESIDENT_ENTRY(ms_resident_pages_r20, ms::kCipherChaCha, 20)
MS_RESIDENT_ENTRY(ms_resident_pages_r12, ms::kCipherChaCha, 12)
MS_RESIDENT_ENTRY(ms_resident_pages_r8, ms::kCipherChaCha, 8)
MS_RESIDENT_ENTRY(ms_resident_pages_s20, ms::kCipherSalsa, 20)
MS_RESIDENT_ENTRY(ms_resident_pages_s12, ms::kCipherSalsa, 12)
MS_RESIDENT_ENTRY(ms_resident_pages_s8, ms::kCipherSalsa, 8)
