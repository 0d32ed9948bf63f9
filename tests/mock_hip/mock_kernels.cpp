// CPU versions of the page kernels' launch functions (ms_kernels.h) for the
// mock HIP runtime: each launch becomes an operation on its stream that
// ciphers the same pages with the same keys and nonces through the C
// oracle (test infrastructure only).  Also weak stubs for the host-page and
// resident-key parts of the library, for a build that leaves them out.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>

#include "ms_internal.h"
#include "ms_kernels.h"

extern "C" void oracle_cipher_page(const uint8_t key[32],
                                   const uint8_t nonce[12], int rounds,
                                   const uint8_t* in, uint8_t* out);
extern "C" void oracle_salsa_cipher_page(const uint8_t key[32],
                                         const uint8_t nonce[12], int rounds,
                                         const uint8_t* in, uint8_t* out);

namespace {

struct MockKernel {
  bool batch;
  uint32_t unroll;
  int rounds;
  uint32_t kind;
  uint32_t cipher;
};

int round_index(int rounds) { return rounds == 8 ? 0 : (rounds == 12 ? 1 : 2); }

MockKernel g_plain[2][3][2][2];
MockKernel g_batch[2][3][2];

struct Init {
  Init() {
    const int rs[3] = {8, 12, 20};
    for (uint32_t c = 0; c < 2; ++c)
      for (int r = 0; r < 3; ++r)
        for (uint32_t u = 0; u < 2; ++u) {
          g_batch[c][r][u] = MockKernel{true, u + 1, rs[r], 0, c};
          for (uint32_t k = 0; k < 2; ++k)
            g_plain[c][r][u][k] = MockKernel{false, u + 1, rs[r], k, c};
        }
  }
} g_init;

void put_le32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
  p[2] = (uint8_t)(v >> 16);
  p[3] = (uint8_t)(v >> 24);
}

void key_bytes(const uint32_t* keys, uint32_t slot, uint8_t out[32]) {
  for (int i = 0; i < 8; ++i) put_le32(out + 4 * i, keys[(uint64_t)slot * 8 + i]);
}

void cipher(const uint8_t key[32], uint32_t kind, const uint32_t* nonce_array,
            uint64_t nonce_base, uint64_t nonce_stride, uint32_t tag,
            uint64_t i, uint32_t which, int rounds, const uint8_t* src,
            uint8_t* dst) {
  uint8_t n[12];
  if (kind == ms::kNonceArray) {
    for (int w = 0; w < 3; ++w) put_le32(n + 4 * w, nonce_array[i * 3 + w]);
  } else {
    const uint64_t v = nonce_base + i * nonce_stride;
    put_le32(n, (uint32_t)v);
    put_le32(n + 4, (uint32_t)(v >> 32));
    put_le32(n + 8, tag);
  }
  if (which == ms::kCipherSalsa)
    oracle_salsa_cipher_page(key, n, rounds, src + i * ms::kPageBytes,
                             dst + i * ms::kPageBytes);
  else
    oracle_cipher_page(key, n, rounds, src + i * ms::kPageBytes,
                       dst + i * ms::kPageBytes);
}

void run_batch(const ms::DevBatchHdr* hdr, const uint32_t* keys,
               uint32_t which, int rounds) {
  const auto* reqs = reinterpret_cast<const ms::DevReq*>(hdr + 1);
  for (uint32_t r = 0; r < hdr->n_req; ++r) {
    const ms::DevReq& q = reqs[r];
    uint8_t k[32];
    key_bytes(keys, q.key_slot, k);
    for (uint64_t i = 0; i < q.page_end - q.page_begin; ++i)
      cipher(k, q.kind, reinterpret_cast<const uint32_t*>(q.nonce), q.nonce,
             q.stride, q.tag, i, which, rounds,
             reinterpret_cast<const uint8_t*>(q.src),
             reinterpret_cast<uint8_t*>(q.dst));
  }
}

}  // namespace

void mock_run_batch_node(const void* func, const void* hdr,
                         const uint32_t* keys, uint32_t) {
  const auto* k = static_cast<const MockKernel*>(func);
  run_batch(static_cast<const ms::DevBatchHdr*>(hdr), keys, k->cipher,
            k->rounds);
}

namespace ms {

const void* batch_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds) {
  return &g_batch[cipher ? 1 : 0][round_index(rounds)][unroll == 2 ? 1 : 0];
}
const void* plain_kernel_fn(uint32_t unroll, uint32_t cipher, int rounds,
                            uint32_t kind) {
  return &g_plain[cipher ? 1 : 0][round_index(rounds)][unroll == 2 ? 1 : 0]
                 [kind ? 1 : 0];
}
uint32_t resident_waves_per_cu(const void*) { return 28; }

hipError_t launch_plain(const PlainArgs& a, uint32_t kind, uint32_t which,
                        int rounds, uint32_t max_waves, uint32_t unroll,
                        hipStream_t stream) {
  if (max_waves == 0 || (unroll != 1 && unroll != 2)) return hipErrorInvalidValue;
  const PlainArgs x = a;
  mock_enqueue(stream, [x, kind, which, rounds] {
    uint8_t k[32];
    key_bytes(x.keys, x.key_slot, k);
    for (uint64_t i = 0; i < x.n_pages; ++i)
      cipher(k, kind, x.nonce_array, x.nonce_base, x.nonce_stride,
             x.nonce_tag, x.first_page + i, which, rounds, x.src, x.dst);
  });
  return hipSuccess;
}

hipError_t launch_batch(const DevBatchHdr* batch, const uint32_t* keys,
                        uint32_t, uint32_t unroll, uint32_t grid_blocks,
                        uint32_t which, int rounds, hipStream_t stream) {
  if (grid_blocks == 0 || (unroll != 1 && unroll != 2)) return hipErrorInvalidValue;
  mock_enqueue(stream, [batch, keys, which, rounds] {
    run_batch(batch, keys, which, rounds);
  });
  return hipSuccess;
}

hipError_t launch_batch_inline(const InlineBatch& batch, const uint32_t* keys,
                               uint32_t, uint32_t unroll, uint32_t grid_blocks,
                               uint32_t which, int rounds, hipStream_t stream) {
  if (grid_blocks == 0 || (unroll != 1 && unroll != 2) ||
      batch.hdr.n_req == 0 || batch.hdr.n_req > kInlineBatchMax)
    return hipErrorInvalidValue;
  // the arguments are copied at the launch, as the runtime does
  auto copy = std::make_shared<InlineBatch>(batch);
  mock_enqueue(stream, [copy, keys, which, rounds] {
    run_batch(&copy->hdr, keys, which, rounds);
  });
  return hipSuccess;
}

// The device array of the allocation-free batch entry point: host memory
// here, like every mock device buffer.
alignas(256) static uint8_t g_static_scratch[kStaticBatchBytes];

hipError_t static_batch_scratch(void** out) {
  if (!out) return hipErrorInvalidValue;
  *out = g_static_scratch;
  return hipSuccess;
}

// The descriptor copy: a stream-ordered memmove here (graph nodes of it are
// recognised by this entry point in mock_hip.cpp).
static const char g_desc_copy = 0;
const void* desc_copy_fn() { return &g_desc_copy; }
uint32_t desc_copy_blocks(size_t bytes) {
  return (uint32_t)((bytes / 16 + kBlockThreads - 1) / kBlockThreads);
}
hipError_t launch_desc_copy(void* dev, const void* host, size_t bytes,
                            hipStream_t stream) {
  if (!dev || !host || bytes == 0 || bytes % 16 != 0)
    return hipErrorInvalidValue;
  mock_enqueue(stream, [dev, host, bytes] { std::memmove(dev, host, bytes); });
  return hipSuccess;
}

hipError_t launch_copy(const void*, void*, uint64_t, uint32_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_valu(uint32_t*, uint32_t, uint32_t, hipStream_t) {
  return hipErrorInvalidValue;
}
uint64_t valu_probe_ops(uint32_t, uint32_t) { return 0; }
hipError_t launch_fill_u32(uint32_t* dst, uint32_t value, uint64_t n_words,
                           hipStream_t stream) {
  mock_enqueue(stream, [dst, value, n_words] {
    for (uint64_t i = 0; i < n_words; ++i) dst[i] = value;
  });
  return hipSuccess;
}

}  // namespace ms

// Used when host_pages.cpp and resident.cpp are not linked in.
__attribute__((weak)) HostPath* ms_internal_host_path_create() {
  return reinterpret_cast<HostPath*>(new char[1]);
}
__attribute__((weak)) void ms_internal_host_path_destroy(HostPath* h) {
  delete[] reinterpret_cast<char*>(h);
}
__attribute__((weak)) void ms_internal_resident_stop_all(ms_ctx*) {}
__attribute__((weak)) ms_status ms_internal_ring_start(
    ms_ctx*, const ms_resident_config*, const uint32_t*, uint32_t,
    ms_resident**) {
  return MS_ENOTSUP;
}
__attribute__((weak)) ms_status ms_internal_ring_publish(
    ms_resident*, uint32_t, const void*, void*, uint64_t, const ms_nonce&,
    ms_ticket*) {
  return MS_ENOTSUP;
}
__attribute__((weak)) int ms_internal_ring_done(ms_resident*, ms_ticket) {
  return 0;
}
__attribute__((weak)) void ms_internal_ring_span(ms_ticket, uint64_t* first,
                                                 uint64_t* count) {
  *first = 0;
  *count = 0;
}
__attribute__((weak)) uint64_t ms_internal_ring_published(ms_resident*) {
  return 0;
}
__attribute__((weak)) uint64_t ms_internal_ring_advance(ms_resident*,
                                                        uint64_t from,
                                                        uint64_t) {
  return from;
}
__attribute__((weak)) uint32_t ms_internal_resident_live(int) { return 0; }
__attribute__((weak)) bool ms_internal_ring_alive(ms_resident*) {
  return false;
}
__attribute__((weak)) void ms_internal_ring_stop(ms_resident*) {}
__attribute__((weak)) void ms_resident_config_default(ms_resident_config* c) {
  std::memset(c, 0, sizeof(*c));
}
