// Many-thread stress of the engine's serving path on the mock HIP runtime
// (test infrastructure only; built and run under ThreadSanitizer by
// tests/test_scheduler_tsan_cpu.py).
//
// Each request is served alone first (submit, wait), then all of them again
// from 8 submitting threads at once, with prefetch hints beside them and a
// ninth thread that keeps submitting for one client and cancelling it.  The
// configuration is small (queue depth, admission cap, batch size, batch
// slots) so that admission blocking, full queues, batch splitting and the
// scheduler's sleep all happen.  Every mixed result must equal the alone
// result byte for byte, a sample must equal the C oracle, and the fused
// batch of ms_process_batch (graph replay) must agree too.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "memshield.h"

extern "C" void oracle_cipher_page(const uint8_t key[32],
                                   const uint8_t nonce[12], int rounds,
                                   const uint8_t* in, uint8_t* out);

#define CHECK(x)                                                          \
  do {                                                                    \
    const int _s = (int)(x);                                              \
    if (_s != 0) {                                                        \
      std::fprintf(stderr, "FAILED %s -> %d (line %d)\n", #x, _s, __LINE__); \
      return 1;                                                           \
    }                                                                     \
  } while (0)

namespace {

uint64_t rng_state = 0x9E3779B97F4A7C15ull;
uint64_t next_rand() {  // xorshift64*, single-threaded setup only
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545F4914F6CDD1Dull;
}

constexpr int kThreads = 8;
constexpr int kPerThread = 40;
constexpr int kReqs = kThreads * kPerThread;
constexpr int kClients = 12;
constexpr uint32_t kCancelClient = 77;

struct Req {
  uint32_t client;
  uint64_t off;    // first page in the pools
  uint64_t pages;
  uint64_t va;
};

}  // namespace

int main() {
  ms_config cfg;
  ms_config_default(&cfg);
  cfg.queue_depth = 128;
  cfg.max_batch_requests = 16;
  cfg.admission_cap_bytes = 96ull * 4096;
  cfg.inflight_batches = 3;
  cfg.prefetch_depth = 16;
  cfg.serve_spin_us = 300;
#ifdef RING_STAGE
  // the ring serving stage (resident kernel on the mock HSA runtime); a few
  // requests above the ring's page limit still take the fused launches
  cfg.serve_stage = MS_SERVE_STAGE_RING;
#else
  cfg.serve_stage = MS_SERVE_STAGE_LAUNCH;
#endif
  ms_ctx* c = nullptr;
  CHECK(ms_init(&c, 0, &cfg));

  uint8_t kb[kClients][32];
  ms_key keys[kClients];
  for (int i = 0; i < kClients; ++i) {
    for (int j = 0; j < 32; ++j) kb[i][j] = (uint8_t)next_rand();
    CHECK(ms_key_load(c, kb[i], &keys[i]));
  }
  ms_key cancel_key;
  CHECK(ms_key_load(c, kb[0], &cancel_key));

  std::vector<Req> reqs(kReqs);
  uint64_t total = 0;
  for (int i = 0; i < kReqs; ++i) {
    reqs[i].client = (uint32_t)(next_rand() % kClients);
    reqs[i].pages = 1 + next_rand() % 16;
    reqs[i].off = total;
    reqs[i].va = 0x7f0000000000ull + 4096 * (next_rand() % (1u << 20));
    total += reqs[i].pages;
  }
  uint8_t *src, *dst_a, *dst_b, *dst_c, *scratch;
  CHECK(hipMalloc((void**)&src, total * 4096));
  CHECK(hipMalloc((void**)&dst_a, total * 4096));
  CHECK(hipMalloc((void**)&dst_b, total * 4096));
  CHECK(hipMalloc((void**)&dst_c, total * 4096));
  // hint i writes its own 16 pages; the cancelled client's requests (one in
  // flight at a time) write the last 4
  const uint64_t hint_pages = (kReqs / 5 + 1) * 16;
  CHECK(hipMalloc((void**)&scratch, (hint_pages + 4) * 4096));
  std::vector<uint8_t> host(total * 4096);
  for (auto& b : host) b = (uint8_t)next_rand();
  CHECK(hipMemcpy(src, host.data(), host.size(), hipMemcpyHostToDevice));

  auto make = [&](int i, uint8_t* dst) {
    ms_request r;
    std::memset(&r, 0, sizeof(r));
    r.op = i % 2;
    r.client = reqs[i].client;
    r.key = keys[reqs[i].client];
    r.src = src + reqs[i].off * 4096;
    r.dst = dst + reqs[i].off * 4096;
    r.n_pages = reqs[i].pages;
    r.nonce.kind = MS_NONCE_LINEAR;
    r.nonce.base = reqs[i].va;
    r.nonce.stride = 4096;
    r.nonce.tag = 1000 + reqs[i].client;
    return r;
  };

  // 1. alone
  for (int i = 0; i < kReqs; ++i) {
    ms_request r = make(i, dst_a);
    ms_ticket t;
    CHECK(ms_submit(c, &r, 1, &t));
    int32_t d = 0;
    CHECK(ms_poll(c, &t, 1, &d, 60ull * 1000000000ull));
    if (d != 1) { std::fprintf(stderr, "alone %d -> %d\n", i, d); return 1; }
  }

  // 2. the mix, with hints and a cancelled client beside it
  std::vector<ms_ticket> tickets(kReqs);
  std::atomic<int> failures{0};
  std::atomic<bool> mix_done{false};
  std::atomic<uint64_t> retries{0}, hints{0}, cancelled{0};
  auto submitter = [&](int t) {
    for (int i = t; i < kReqs; i += kThreads) {
      ms_request r = make(i, dst_b);
      for (;;) {
        const ms_status s = ms_submit(c, &r, 1, &tickets[i]);
        if (s == MS_OK) break;
        if (s != MS_EAGAIN) { failures.fetch_add(1); return; }
        retries.fetch_add(1);
        std::this_thread::yield();
      }
      if (i % 5 == 0) {
        ms_request h = make(i, scratch);
        h.dst = scratch + (uint64_t)(i / 5) * 16 * 4096;
        ms_ticket ht;
        if (ms_prefetch_hint(c, &h, 1, &ht) != MS_OK) failures.fetch_add(1);
        hints.fetch_add(1);
      }
    }
  };
  auto canceller = [&]() {
    while (!mix_done.load()) {
      ms_request r = make(0, scratch);
      r.client = kCancelClient;
      r.key = cancel_key;
      r.src = src;
      r.dst = scratch + hint_pages * 4096;
      r.n_pages = 4;
      ms_ticket t;
      const ms_status s = ms_submit(c, &r, 1, &t);
      if (s == MS_EAGAIN) {
        std::this_thread::yield();
        continue;
      }
      if (s != MS_OK) { failures.fetch_add(1); return; }
      uint64_t n = 0;
      if (ms_cancel_client(c, kCancelClient, &n) != MS_OK) failures.fetch_add(1);
      cancelled.fetch_add(n);
      // cancelled, or launched before the cancel and then completed; wait
      // for it before reusing its destination
      int32_t d = 0;
      if (ms_poll(c, &t, 1, &d, 60ull * 1000000000ull) != MS_OK ||
          (d != 1 && d != MS_ECANCELED))
        failures.fetch_add(1);
    }
  };
  std::thread cancel_thread(canceller);
  std::vector<std::thread> th;
  for (int t = 0; t < kThreads; ++t) th.emplace_back(submitter, t);
  for (auto& x : th) x.join();
  std::vector<int32_t> done(kReqs);
  const ms_status ps =
      ms_poll(c, tickets.data(), kReqs, done.data(), 60ull * 1000000000ull);
  mix_done.store(true);
  cancel_thread.join();
  CHECK(ps);
  CHECK(failures.load());
  for (int i = 0; i < kReqs; ++i)
    if (done[i] != 1) { std::fprintf(stderr, "mix %d -> %d\n", i, done[i]); return 1; }
  CHECK(ms_drain(c, 60ull * 1000000000ull));

  // 3. alone == mix, and alone == the oracle on a sample
  std::vector<uint8_t> a(total * 4096), b(total * 4096);
  CHECK(hipMemcpy(a.data(), dst_a, a.size(), hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(b.data(), dst_b, b.size(), hipMemcpyDeviceToHost));
  if (std::memcmp(a.data(), b.data(), a.size()) != 0) {
    std::fprintf(stderr, "mix differs from alone\n");
    return 1;
  }
  for (int i = 0; i < kReqs; i += 7) {
    for (uint64_t p = 0; p < reqs[i].pages; ++p) {
      uint8_t n[12], want[4096];
      const uint64_t v = reqs[i].va + 4096 * p;
      for (int k = 0; k < 8; ++k) n[k] = (uint8_t)(v >> (8 * k));
      const uint32_t tag = 1000 + reqs[i].client;
      for (int k = 0; k < 4; ++k) n[8 + k] = (uint8_t)(tag >> (8 * k));
      const uint64_t off = (reqs[i].off + p) * 4096;
      oracle_cipher_page(kb[reqs[i].client], n, 20, host.data() + off, want);
      if (std::memcmp(want, a.data() + off, 4096) != 0) {
        std::fprintf(stderr, "request %d page %lu differs from the oracle\n",
                     i, (unsigned long)p);
        return 1;
      }
    }
  }

  // 4. the fused batch (graph replay) agrees
  for (int base = 0; base + 16 <= 64; base += 16) {
    std::vector<ms_request> batch;
    for (int i = base; i < base + 16; ++i) batch.push_back(make(i, dst_c));
    CHECK(ms_process_batch(c, batch.data(), batch.size(), nullptr));
  }
  CHECK(hipDeviceSynchronize());
  std::vector<uint8_t> cc(reqs[64].off * 4096);
  CHECK(hipMemcpy(cc.data(), dst_c, cc.size(), hipMemcpyDeviceToHost));
  if (std::memcmp(cc.data(), a.data(), cc.size()) != 0) {
    std::fprintf(stderr, "fused batch differs from alone\n");
    return 1;
  }

  ms_stats st;
  CHECK(ms_get_stats(c, &st));
  CHECK(ms_shutdown(c));
  std::printf("ok requests=%d batches=%lu eagain_retries=%lu hints=%lu "
              "cancelled=%lu max_batch=%lu max_inflight_batches=%lu\n",
              kReqs, (unsigned long)st.batches, (unsigned long)retries.load(),
              (unsigned long)hints.load(), (unsigned long)cancelled.load(),
              (unsigned long)st.max_batch_requests,
              (unsigned long)st.max_inflight_batches);
  for (auto* p : {src, dst_a, dst_b, dst_c, scratch}) CHECK(hipFree(p));
  return 0;
}
