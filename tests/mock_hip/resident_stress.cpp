// Many-thread stress of the resident-key engine's host side (resident.cpp,
// with host_pages.cpp and engine.cpp) on the mock HIP and HSA runtimes, whose
// CPU model of the resident kernel keeps its protocol (test infrastructure
// only; built and run under ThreadSanitizer by
// tests/test_resident_tsan_cpu.py).
//
// 1. A five-key engine with a small ring (64 positions, 2 pages a
//    descriptor): 6 producer threads each submit 40 requests of 1..9 pages
//    with a random key, linear or array nonces, device or pinned host pages,
//    in place or not, keeping up to 4 in flight and retrying on MS_EAGAIN,
//    so that slots are reused under contention; every result must equal the
//    C oracle.  The key buffer must read wiped once the engine is up.
// 2. An engine with an idle limit: it serves a request, then ends by itself;
//    alive reads 0, a submission returns MS_ECLOSED, the old ticket still
//    reads done, stop succeeds.
// 3. An engine with a key from the OS CSPRNG, at 8 rounds: encrypting twice
//    gives the pages back.
// 4. An engine left running is stopped by ms_shutdown.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "memshield.h"
#include "memshield_host.h"
#include "memshield_resident.h"

extern "C" void oracle_cipher_page(const uint8_t key[32],
                                   const uint8_t nonce[12], int rounds,
                                   const uint8_t* in, uint8_t* out);

#define CHECK(x)                                                             \
  do {                                                                       \
    const int _s = (int)(x);                                                 \
    if (_s != 0) {                                                           \
      std::fprintf(stderr, "FAILED %s -> %d (line %d)\n", #x, _s, __LINE__); \
      return 1;                                                              \
    }                                                                        \
  } while (0)

namespace {

constexpr uint64_t kPage = 4096;
constexpr int kProducers = 6;
constexpr int kPerProducer = 40;
constexpr int kReqs = kProducers * kPerProducer;
constexpr uint32_t kKeys = 5;
constexpr int kWindow = 4;
constexpr uint64_t kWaitNs = 60ull * 1000000000ull;

uint64_t rng_state = 0x243F6A8885A308D3ull;
uint64_t next_rand() {  // xorshift64*, single-threaded setup only
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545F4914F6CDD1Dull;
}

void put_le32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

struct Req {
  uint64_t off;   // first page in the pools
  uint64_t pages;
  uint32_t key;
  bool array;     // nonce array, else linear
  bool host;      // pinned host pools, else device pools
  bool in_place;
  uint64_t va;
  uint32_t tag;
};

// The pools of one memory kind: plaintext, output, and per-page nonces.
struct Pools {
  uint8_t* src;
  uint8_t* dst;
  uint8_t* nonces;
};

}  // namespace

int main() {
  ms_config cfg;
  ms_config_default(&cfg);
  ms_ctx* c = nullptr;
  CHECK(ms_init(&c, 0, &cfg));
  const int rounds = 20;

  // ---- 1. five keys, six producers, a small ring
  uint8_t kb[kKeys][32];
  ms_key handles[kKeys];
  for (uint32_t i = 0; i < kKeys; ++i) {
    for (int j = 0; j < 32; ++j) kb[i][j] = (uint8_t)next_rand();
    CHECK(ms_key_load(c, kb[i], &handles[i]));
  }
  std::vector<Req> reqs(kReqs);
  uint64_t total = 0;
  for (int i = 0; i < kReqs; ++i) {
    Req& q = reqs[i];
    q.off = total;
    q.pages = 1 + next_rand() % 9;
    q.key = (uint32_t)(next_rand() % kKeys);
    q.array = next_rand() % 2;
    q.host = next_rand() % 3 == 0;
    q.in_place = next_rand() % 4 == 0;
    q.va = 0x7f0000000000ull + kPage * (next_rand() % (1u << 20));
    q.tag = (uint32_t)next_rand();
    total += q.pages;
  }
  std::vector<uint8_t> plain(total * kPage), nonce_bytes(total * 12);
  for (auto& b : plain) b = (uint8_t)next_rand();
  for (auto& b : nonce_bytes) b = (uint8_t)next_rand();
  Pools dev{}, host{};
  CHECK(hipMalloc((void**)&dev.src, total * kPage));
  CHECK(hipMalloc((void**)&dev.dst, total * kPage));
  CHECK(hipMalloc((void**)&dev.nonces, total * 12));
  CHECK(ms_host_alloc(c, total * kPage, (void**)&host.src));
  CHECK(ms_host_alloc(c, total * kPage, (void**)&host.dst));
  CHECK(ms_host_alloc(c, total * 12, (void**)&host.nonces));
  for (Pools* p : {&dev, &host}) {
    CHECK(hipMemcpy(p->src, plain.data(), plain.size(), hipMemcpyHostToDevice));
    // in-place requests start from the plaintext in the output pool
    CHECK(hipMemcpy(p->dst, plain.data(), plain.size(), hipMemcpyHostToDevice));
    CHECK(hipMemcpy(p->nonces, nonce_bytes.data(), nonce_bytes.size(),
                    hipMemcpyHostToDevice));
  }

  ms_resident_config rc;
  ms_resident_config_default(&rc);
  rc.workers = 23;
  rc.ring_depth = 64;
  rc.desc_pages = 2;
  rc.idle_limit_ms = 0;
  ms_resident* r = nullptr;
  CHECK(ms_resident_start_keys(c, &rc, handles, kKeys, &r));
  if (ms_resident_alive(r) != 1 || ms_resident_debug_key_wiped(r) != 1) {
    std::fprintf(stderr, "engine not up, or its key buffer not wiped\n");
    return 1;
  }

  std::atomic<int> failures{0};
  std::atomic<uint64_t> retries{0};
  auto producer = [&](int t) {
    std::vector<ms_ticket> window;
    auto drain = [&]() {
      if (window.empty()) return;
      std::vector<int32_t> done(window.size());
      if (ms_resident_poll(r, window.data(), window.size(), done.data(), kWaitNs) != MS_OK)
        failures.fetch_add(1);
      for (int32_t d : done)
        if (d != 1) failures.fetch_add(1);
      window.clear();
    };
    for (int i = t; i < kReqs; i += kProducers) {
      const Req& q = reqs[i];
      const Pools& p = q.host ? host : dev;
      ms_nonce n;
      std::memset(&n, 0, sizeof(n));
      if (q.array) {
        n.kind = MS_NONCE_ARRAY;
        n.array = p.nonces + q.off * 12;
      } else {
        n.kind = MS_NONCE_LINEAR;
        n.base = q.va;
        n.stride = kPage;
        n.tag = q.tag;
      }
      uint8_t* dst = p.dst + q.off * kPage;
      const uint8_t* src = q.in_place ? dst : p.src + q.off * kPage;
      ms_ticket tk;
      for (;;) {
        const ms_status s = ms_resident_submit_keyed(r, q.key, src, dst, q.pages, &n, &tk);
        if (s == MS_OK) break;
        if (s != MS_EAGAIN) {
          std::fprintf(stderr, "submit %d -> %d\n", i, (int)s);
          failures.fetch_add(1);
          return;
        }
        retries.fetch_add(1);
        std::this_thread::yield();
      }
      window.push_back(tk);
      if (window.size() == kWindow) drain();
    }
    drain();
  };
  std::vector<std::thread> th;
  for (int t = 0; t < kProducers; ++t) th.emplace_back(producer, t);
  for (auto& x : th) x.join();
  CHECK(failures.load());

  std::vector<uint8_t> out_dev(total * kPage), out_host(total * kPage);
  CHECK(hipMemcpy(out_dev.data(), dev.dst, out_dev.size(), hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(out_host.data(), host.dst, out_host.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < kReqs; ++i) {
    const Req& q = reqs[i];
    const uint8_t* got = (q.host ? out_host : out_dev).data();
    for (uint64_t p = 0; p < q.pages; ++p) {
      const uint64_t page = q.off + p;
      uint8_t n[12], want[kPage];
      if (q.array) {
        std::memcpy(n, nonce_bytes.data() + page * 12, 12);
      } else {
        const uint64_t v = q.va + p * kPage;
        put_le32(n, (uint32_t)v);
        put_le32(n + 4, (uint32_t)(v >> 32));
        put_le32(n + 8, q.tag);
      }
      oracle_cipher_page(kb[q.key], n, rounds, plain.data() + page * kPage, want);
      if (std::memcmp(want, got + page * kPage, kPage) != 0) {
        std::fprintf(stderr, "request %d page %lu differs from the oracle\n", i,
                     (unsigned long)p);
        return 1;
      }
    }
  }
  CHECK(ms_resident_stop(r));

  // ---- 2. an idle limit: the engine ends by itself
  rc.workers = 3;
  rc.ring_depth = 16;
  rc.desc_pages = 4;
  rc.idle_limit_ms = 30;
  CHECK(ms_resident_start(c, &rc, kb[1], &r));
  ms_nonce lin;
  std::memset(&lin, 0, sizeof(lin));
  lin.kind = MS_NONCE_LINEAR;
  lin.base = 0x1000;
  lin.stride = kPage;
  lin.tag = 9;
  ms_ticket tk;
  CHECK(ms_resident_submit(r, dev.src, dev.dst, 5, &lin, &tk));
  int32_t d = 0;
  CHECK(ms_resident_poll(r, &tk, 1, &d, kWaitNs));
  if (d != 1) { std::fprintf(stderr, "idle engine: request not done\n"); return 1; }
  const auto t0 = std::chrono::steady_clock::now();
  while (ms_resident_alive(r)) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(30)) {
      std::fprintf(stderr, "idle engine did not end\n");
      return 1;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(5));
  }
  const ms_status closed = ms_resident_submit(r, dev.src, dev.dst, 1, &lin, nullptr);
  if (closed != MS_ECLOSED) { std::fprintf(stderr, "closed -> %d\n", (int)closed); return 1; }
  CHECK(ms_resident_poll(r, &tk, 1, &d, 0));
  if (d != 1) { std::fprintf(stderr, "old ticket after idle exit -> %d\n", d); return 1; }
  CHECK(ms_resident_stop(r));

  // ---- 3. a key from the OS CSPRNG at 8 rounds: twice is the identity
  ms_ctx* c8 = nullptr;
  ms_config cfg8 = cfg;
  cfg8.rounds = 8;
  CHECK(ms_init(&c8, 0, &cfg8));
  rc.workers = 5;
  rc.idle_limit_ms = 0;
  CHECK(ms_resident_start(c8, &rc, nullptr, &r));
  ms_ticket t1, t2;
  CHECK(ms_resident_submit(r, dev.src, dev.dst, 9, &lin, &t1));
  CHECK(ms_resident_poll(r, &t1, 1, &d, kWaitNs));
  CHECK(ms_resident_submit(r, dev.dst, dev.dst, 9, &lin, &t2));
  CHECK(ms_resident_poll(r, &t2, 1, &d, kWaitNs));
  std::vector<uint8_t> back(9 * kPage);
  CHECK(hipMemcpy(back.data(), dev.dst, back.size(), hipMemcpyDeviceToHost));
  if (std::memcmp(back.data(), plain.data(), back.size()) != 0) {
    std::fprintf(stderr, "random-key round trip differs\n");
    return 1;
  }
  CHECK(ms_resident_stop(r));
  CHECK(ms_shutdown(c8));

  // ---- 4. shutdown stops an engine still running, from another thread
  CHECK(ms_resident_start(c, &rc, kb[2], &r));
  CHECK(ms_resident_submit(r, dev.src, dev.dst, 3, &lin, &tk));
  CHECK(ms_resident_poll(r, &tk, 1, &d, kWaitNs));
  ms_status down = MS_EINVAL;
  std::thread closer([&] { down = ms_shutdown(c); });
  closer.join();
  CHECK(down);

  CHECK(hipFree(dev.src));
  CHECK(hipFree(dev.dst));
  CHECK(hipFree(dev.nonces));
  std::printf("ok requests=%d eagain_retries=%lu\n", kReqs,
              (unsigned long)retries.load());
  return 0;
}
