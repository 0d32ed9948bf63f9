// Key destroy and reload racing synchronous calls, on the mock HIP runtime
// (test infrastructure only; built and run under ThreadSanitizer by
// tests/test_scheduler_tsan_cpu.py).
//
// The context has room for two keys, so a destroyed row is the one the next
// load takes.  One thread keeps ciphering a page with key A through the
// synchronous calls (ms_encrypt_pages, ms_process_batch, and
// ms_encrypt_host_pages on pinned host pages), always with the newest handle
// of A.  Another thread keeps destroying that handle, loading key B into the
// freed row, destroying B and loading A again.  A call may fail with
// MS_ENOKEY (its handle went stale) and a destroy with MS_EBUSY (a call held
// the row), but every call that returns MS_OK must have ciphered with key A:
// its page must equal the C oracle under A.  A call that resolved A's handle
// and then launched after the row was wiped and refilled with B would write
// B's ciphertext (or the zero key's).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "memshield.h"
#include "memshield_host.h"

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

int main() {
  ms_config cfg;
  ms_config_default(&cfg);
  cfg.max_keys = 2;
  cfg.queue_depth = 64;
  cfg.max_batch_requests = 8;
  ms_ctx* c = nullptr;
  CHECK(ms_init(&c, 0, &cfg));

  uint8_t key_a[32], key_b[32], page[4096], want[4096], nonce_b[12];
  for (int i = 0; i < 32; ++i) {
    key_a[i] = (uint8_t)(3 * i + 1);
    key_b[i] = (uint8_t)(200 - 5 * i);
  }
  for (int i = 0; i < 4096; ++i) page[i] = (uint8_t)(i * 7 + 11);
  const uint64_t va = 0x7f0000123000ull;
  const uint32_t pid = 4321;
  for (int k = 0; k < 8; ++k) nonce_b[k] = (uint8_t)(va >> (8 * k));
  for (int k = 0; k < 4; ++k) nonce_b[8 + k] = (uint8_t)(pid >> (8 * k));
  oracle_cipher_page(key_a, nonce_b, 20, page, want);

  uint8_t *src, *dst;
  CHECK(hipMalloc((void**)&src, 4096));
  CHECK(hipMalloc((void**)&dst, 4096));
  CHECK(hipMemcpy(src, page, 4096, hipMemcpyHostToDevice));
  uint8_t *hsrc = nullptr, *hdst = nullptr;
  CHECK(ms_host_alloc(c, 4096, (void**)&hsrc));
  CHECK(ms_host_alloc(c, 4096, (void**)&hdst));
  std::memcpy(hsrc, page, 4096);

  ms_key first;
  CHECK(ms_key_load(c, key_a, &first));
  std::atomic<uint64_t> handle_a{first};
  std::atomic<bool> done{false};
  std::atomic<int> failures{0};
  std::atomic<uint64_t> ok_calls{0}, stale{0}, busy{0}, cycles{0};

  auto caller = [&]() {
    ms_nonce n;
    std::memset(&n, 0, sizeof(n));
    n.kind = MS_NONCE_LINEAR;
    n.base = va;
    n.stride = 4096;
    n.tag = pid;
    uint8_t got[4096];
    for (int it = 0; it < 3000; ++it) {
      const ms_key k = handle_a.load();
      const int kind = it % 3;
      ms_status s;
      if (kind == 0) {
        if (hipMemset(dst, 0, 4096) != hipSuccess) { failures++; return; }
        s = ms_encrypt_pages(c, k, src, dst, 1, &n, nullptr);
      } else if (kind == 1) {
        if (hipMemset(dst, 0, 4096) != hipSuccess) { failures++; return; }
        ms_request r;
        std::memset(&r, 0, sizeof(r));
        r.op = MS_ENCRYPT;
        r.key = k;
        r.src = src;
        r.dst = dst;
        r.n_pages = 1;
        r.nonce = n;
        s = ms_process_batch(c, &r, 1, nullptr);
      } else {
        std::memset(hdst, 0, 4096);
        s = ms_encrypt_host_pages(c, k, hsrc, hdst, 1, &n, MS_HOST_MAPPED,
                                  nullptr);
      }
      if (s == MS_ENOKEY) {
        stale++;
        continue;
      }
      if (s != MS_OK) {
        std::fprintf(stderr, "call kind %d -> %d\n", kind, (int)s);
        failures++;
        return;
      }
      if (hipDeviceSynchronize() != hipSuccess) { failures++; return; }
      if (kind == 2) {
        std::memcpy(got, hdst, 4096);
      } else if (hipMemcpy(got, dst, 4096, hipMemcpyDeviceToHost) !=
                 hipSuccess) {
        failures++;
        return;
      }
      if (std::memcmp(got, want, 4096) != 0) {
        std::fprintf(stderr, "call kind %d (iteration %d) did not cipher "
                     "with key A\n", kind, it);
        failures++;
        return;
      }
      ok_calls++;
    }
  };

  auto rotator = [&]() {
    while (!done.load()) {
      const ms_key k = handle_a.load();
      const ms_status s = ms_key_destroy(c, k);
      if (s == MS_EBUSY) {
        busy++;
        std::this_thread::yield();
        continue;
      }
      if (s != MS_OK) { failures++; return; }
      ms_key kb, ka;
      // the freed row takes B, then A again in a row of its own choosing
      if (ms_key_load(c, key_b, &kb) != MS_OK) { failures++; return; }
      if (ms_key_destroy(c, kb) != MS_OK) { failures++; return; }
      if (ms_key_load(c, key_a, &ka) != MS_OK) { failures++; return; }
      handle_a.store(ka);
      cycles++;
      // give the caller a turn with the fresh handle (on a loaded machine a
      // rotator that never yields can keep every handle it reads stale)
      std::this_thread::yield();
    }
  };

  std::thread rot(rotator);
  std::thread call(caller);
  call.join();
  done.store(true);
  rot.join();
  CHECK(failures.load());
  if (ok_calls.load() == 0) {
    std::fprintf(stderr, "no call completed\n");
    return 1;
  }
  CHECK(ms_host_free(c, hsrc));
  CHECK(ms_host_free(c, hdst));
  CHECK(hipFree(src));
  CHECK(hipFree(dst));
  CHECK(ms_shutdown(c));
  std::printf("ok calls=%lu stale=%lu busy=%lu cycles=%lu\n",
              (unsigned long)ok_calls.load(), (unsigned long)stale.load(),
              (unsigned long)busy.load(), (unsigned long)cycles.load());
  return 0;
}
