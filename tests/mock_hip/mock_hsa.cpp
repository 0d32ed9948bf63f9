// CPU implementation of the mock HSA runtime of hsa/hsa.h, and a CPU model of
// the resident-key kernel that a dispatch packet on a mock queue starts
// (test infrastructure only).
//
// The model keeps the kernel's protocol with the host: one poller thread
// mirrors the host's published count into the device control block and
// leaves on `stop` or after the idle limit (100 MHz ticks, host heartbeats
// counting as activity), then raises the device `stop` and the host
// `exited`; n_workers worker threads take the keys, count themselves in
// `key_loads` (the last wipes the key buffer and raises `ready`), serve the
// ring positions congruent to worker * inv_step modulo n_workers, check
// each descriptor as the kernel does, cipher its pages through the C oracle
// and write the slot's completion word.  When every thread has left, the
// completion signal drops to 0.  Each ordering the kernel gets from its
// waits and system-scope accesses is taken here as an acquire load or a
// release store, so what ThreadSanitizer checks is the host side.
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ms_kernels.h"
#include "ms_resident_kernel.h"

extern "C" void oracle_cipher_page(const uint8_t key[32],
                                   const uint8_t nonce[12], int rounds,
                                   const uint8_t* in, uint8_t* out);

// The engine checks that the code object it loads is this one.
extern "C" const unsigned char ms_resident_code_object[] = {0x7f, 'M', 'O', 'C', 'K'};
extern "C" const size_t ms_resident_code_object_size = sizeof(ms_resident_code_object);

namespace {

using Clock = std::chrono::steady_clock;

template <class T>
T load_acq(const T* p) {
  return __atomic_load_n(p, __ATOMIC_ACQUIRE);
}
template <class T>
void store_rel(T* p, T v) {
  __atomic_store_n(p, v, __ATOMIC_RELEASE);
}

uint64_t ticks_100mhz() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             Clock::now().time_since_epoch())
             .count() /
         10;
}

constexpr uint64_t kCpuAgent = 1, kGpuAgent = 2;
constexpr uint32_t kBus = 0x42;  // the mock HIP device's PCI bus
constexpr uint32_t kGroupBytes = 18432;
constexpr uint64_t kExecutable = 0xE0, kReader = 0xC0;

std::mutex g_mu;  // hsa_init count, live executables and readers
int g_init = 0;

struct MockQueue;

struct MockSignal {
  std::atomic<int64_t> v;
  MockQueue* doorbell_of = nullptr;
};

MockSignal* sig(hsa_signal_t s) { return reinterpret_cast<MockSignal*>(s.handle); }

struct MockQueue {
  hsa_queue_t q{};
  std::atomic<uint64_t> write_index{0};
  hsa_kernel_dispatch_packet_t* packets = nullptr;
  MockSignal doorbell;
  std::thread launcher;  // runs one dispatch: the model's threads, then the signal
};

void put_le32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

struct Model {
  ms::RkArgs a;
  int rounds;

  void poller() {
    uint64_t last_pub = 0, last_hb = 0, t_last = ticks_100mhz();
    for (;;) {
      if (load_acq(&a.hctl->stop)) break;
      const uint64_t pub = load_acq(&a.hctl->published);
      const uint64_t hb = load_acq(&a.hctl->heartbeat);
      const uint64_t now = ticks_100mhz();
      if (pub != last_pub) {
        store_rel(&a.dctl->published, pub);
        last_pub = pub;
        t_last = now;
      } else if (hb != last_hb) {
        last_hb = hb;
        t_last = now;
      } else if (a.idle_ticks != 0 && now - t_last > a.idle_ticks) {
        break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
    store_rel(&a.dctl->stop, 1u);
    store_rel(&a.hctl->exited, 1u);
  }

  void serve_one(const std::vector<uint8_t>& keys, uint64_t pos) {
    const ms::RkDesc d = a.ring[pos & a.ring_mask];
    const uint32_t key_limit = a.n_keys ? a.n_keys : a.table_rows;
    if (d.seq != pos || d.n_pages == 0 || d.n_pages > a.max_pages ||
        d.key >= key_limit || d.kind > 1) {
      store_rel(&a.hctl->error, 1u);
    } else {
      uint8_t row[32];
      const uint8_t* k = keys.data() + (size_t)d.key * 32;
      if (a.n_keys == 0) {
        // a row of the context's key table, read for this descriptor
        for (int i = 0; i < 8; ++i)
          put_le32(row + 4 * i, a.key_table[(size_t)d.key * 8 + i]);
        k = row;
      }
      for (uint32_t p = 0; p < d.n_pages; ++p) {
        uint8_t n[12];
        if (d.kind == 0) {
          std::memcpy(n, reinterpret_cast<const uint8_t*>(d.nonce_base) + 12 * p, 12);
        } else {
          const uint64_t v = d.nonce_base + p * d.nonce_stride;
          put_le32(n, (uint32_t)v);
          put_le32(n + 4, (uint32_t)(v >> 32));
          put_le32(n + 8, d.tag);
        }
        // in place or not, the kernel reads a page whole before writing it
        uint8_t in[ms::kPageBytes], out[ms::kPageBytes];
        std::memcpy(in, reinterpret_cast<const uint8_t*>(d.src) + p * ms::kPageBytes,
                    sizeof(in));
        oracle_cipher_page(k, n, rounds, in, out);
        std::memcpy(reinterpret_cast<uint8_t*>(d.dst) + p * ms::kPageBytes, out,
                    sizeof(out));
      }
    }
    store_rel(&a.completed[pos & a.ring_mask], pos + 1);
  }

  void worker(uint32_t w) {
    // the keys as bytes (little-endian words), from the key buffer
    std::vector<uint8_t> keys((size_t)a.n_keys * 32);
    for (uint32_t i = 0; i < a.n_keys * 8; ++i) put_le32(&keys[4 * i], a.key_buf[i]);
    const uint32_t before =
        __atomic_fetch_add(&a.dctl->key_loads, 1u, __ATOMIC_ACQ_REL);
    if (before + 1 == a.n_workers) {
      for (uint32_t i = 0; i < a.n_keys * 8; ++i) a.key_buf[i] = 0;
      store_rel(&a.hctl->ready, 1u);
    }
    const uint32_t first = (uint32_t)(((uint64_t)w * a.inv_step) % a.n_workers);
    for (uint64_t pos = first;; pos += a.n_workers) {
      if (load_acq(&a.dctl->stop)) return;
      for (;;) {
        const uint64_t pub = load_acq(&a.dctl->published);
        if (pos < pub) break;
        if (load_acq(&a.dctl->stop)) return;
        if (pos == pub)
          std::this_thread::yield();
        else
          std::this_thread::sleep_for(std::chrono::microseconds(pos - pub < 64 ? 10 : 50));
      }
      serve_one(keys, pos);
    }
  }
};

void run_dispatch(MockQueue* mq, uint64_t index) {
  hsa_kernel_dispatch_packet_t* pkt = mq->packets + (index & (mq->q.size - 1));
  const uint32_t hs = __atomic_load_n(reinterpret_cast<uint32_t*>(pkt), __ATOMIC_ACQUIRE);
  const uint16_t header = (uint16_t)hs;
  if (((header >> HSA_PACKET_HEADER_TYPE) & 0xff) != HSA_PACKET_TYPE_KERNEL_DISPATCH ||
      (pkt->kernel_object >> 8) != 1 || pkt->workgroup_size_x != ms::kBlockThreads ||
      pkt->grid_size_x % ms::kBlockThreads || pkt->group_segment_size != kGroupBytes) {
    std::abort();  // a packet the engine never writes
  }
  Model m;
  std::memcpy(&m.a, pkt->kernarg_address, sizeof(m.a));
  m.rounds = (int)(pkt->kernel_object & 0xff);
  const uint32_t waves = pkt->grid_size_x / ms::kWave;
  if (m.a.n_workers + 1 > waves || m.a.n_workers == 0) std::abort();
  const hsa_signal_t done = pkt->completion_signal;
  std::vector<std::thread> th;
  th.emplace_back([&m] { m.poller(); });
  for (uint32_t w = 0; w < m.a.n_workers; ++w) th.emplace_back([&m, w] { m.worker(w); });
  for (auto& t : th) t.join();
  sig(done)->v.fetch_sub(1, std::memory_order_acq_rel);
}

}  // namespace

hsa_status_t hsa_init() {
  std::lock_guard<std::mutex> lk(g_mu);
  ++g_init;
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_shut_down() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_init == 0) return HSA_STATUS_ERROR;
  --g_init;
  return HSA_STATUS_SUCCESS;
}

hsa_status_t hsa_iterate_agents(hsa_status_t (*cb)(hsa_agent_t, void*), void* data) {
  for (uint64_t h : {kCpuAgent, kGpuAgent}) {
    const hsa_status_t s = cb(hsa_agent_t{h}, data);
    if (s != HSA_STATUS_SUCCESS) return s;
  }
  return HSA_STATUS_SUCCESS;
}

hsa_status_t hsa_agent_get_info(hsa_agent_t a, hsa_agent_info_t attr, void* value) {
  if (a.handle != kCpuAgent && a.handle != kGpuAgent) return HSA_STATUS_ERROR;
  switch ((int)attr) {
    case HSA_AGENT_INFO_DEVICE:
      *static_cast<hsa_device_type_t*>(value) =
          a.handle == kGpuAgent ? HSA_DEVICE_TYPE_GPU : HSA_DEVICE_TYPE_CPU;
      return HSA_STATUS_SUCCESS;
    case HSA_AGENT_INFO_QUEUE_MIN_SIZE:
      *static_cast<uint32_t*>(value) = 128;
      return HSA_STATUS_SUCCESS;
    case HSA_AMD_AGENT_INFO_BDFID:
      *static_cast<uint32_t*>(value) = a.handle == kGpuAgent ? kBus << 8 : 0;
      return HSA_STATUS_SUCCESS;
    case HSA_AMD_AGENT_INFO_DOMAIN:
      *static_cast<uint32_t*>(value) = 0;
      return HSA_STATUS_SUCCESS;
  }
  return HSA_STATUS_ERROR;
}

hsa_status_t hsa_code_object_reader_create_from_memory(const void* code, size_t size,
                                                       hsa_code_object_reader_t* r) {
  if (code != ms_resident_code_object || size != ms_resident_code_object_size)
    return HSA_STATUS_ERROR;
  r->handle = kReader;
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_code_object_reader_destroy(hsa_code_object_reader_t r) {
  return r.handle == kReader ? HSA_STATUS_SUCCESS : HSA_STATUS_ERROR;
}
hsa_status_t hsa_executable_create_alt(hsa_profile_t, hsa_default_float_rounding_mode_t,
                                       const char*, hsa_executable_t* e) {
  e->handle = kExecutable;
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_executable_load_agent_code_object(hsa_executable_t e, hsa_agent_t a,
                                                   hsa_code_object_reader_t r,
                                                   const char*, void*) {
  return e.handle == kExecutable && a.handle == kGpuAgent && r.handle == kReader
             ? HSA_STATUS_SUCCESS
             : HSA_STATUS_ERROR;
}
hsa_status_t hsa_executable_freeze(hsa_executable_t e, const char*) {
  return e.handle == kExecutable ? HSA_STATUS_SUCCESS : HSA_STATUS_ERROR;
}
hsa_status_t hsa_executable_get_symbol_by_name(hsa_executable_t e, const char* name,
                                               const hsa_agent_t* a,
                                               hsa_executable_symbol_t* s) {
  if (e.handle != kExecutable || !a || a->handle != kGpuAgent) return HSA_STATUS_ERROR;
  const std::string n(name);
  if (n == ms::kResidentKernel20) s->handle = 20;
  else if (n == ms::kResidentKernel12) s->handle = 12;
  else if (n == ms::kResidentKernel8) s->handle = 8;
  else return HSA_STATUS_ERROR;
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_executable_symbol_get_info(hsa_executable_symbol_t s,
                                            hsa_executable_symbol_info_t attr, void* value) {
  switch (attr) {
    case HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT:
      *static_cast<uint64_t*>(value) = 0x100 | s.handle;  // the round count
      return HSA_STATUS_SUCCESS;
    case HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE:
      *static_cast<uint32_t*>(value) = sizeof(ms::RkArgs);
      return HSA_STATUS_SUCCESS;
    case HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE:
      *static_cast<uint32_t*>(value) = kGroupBytes;
      return HSA_STATUS_SUCCESS;
    case HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE:
      *static_cast<uint32_t*>(value) = 0;
      return HSA_STATUS_SUCCESS;
  }
  return HSA_STATUS_ERROR;
}
hsa_status_t hsa_executable_destroy(hsa_executable_t e) {
  return e.handle == kExecutable ? HSA_STATUS_SUCCESS : HSA_STATUS_ERROR;
}

hsa_status_t hsa_queue_create(hsa_agent_t a, uint32_t size, hsa_queue_type32_t,
                              void (*)(hsa_status_t, hsa_queue_t*, void*), void*,
                              uint32_t, uint32_t, hsa_queue_t** q) {
  if (a.handle != kGpuAgent || size == 0 || (size & (size - 1))) return HSA_STATUS_ERROR;
  auto* mq = new MockQueue();
  mq->packets = static_cast<hsa_kernel_dispatch_packet_t*>(
      std::aligned_alloc(64, size * sizeof(hsa_kernel_dispatch_packet_t)));
  std::memset(mq->packets, 0, size * sizeof(hsa_kernel_dispatch_packet_t));
  mq->doorbell.v.store(-1);
  mq->doorbell.doorbell_of = mq;
  mq->q.base_address = mq->packets;
  mq->q.size = size;
  mq->q.doorbell_signal.handle = reinterpret_cast<uint64_t>(&mq->doorbell);
  mq->q.id = reinterpret_cast<uint64_t>(mq);
  *q = &mq->q;
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_queue_destroy(hsa_queue_t* q) {
  auto* mq = reinterpret_cast<MockQueue*>(q->id);
  if (mq->launcher.joinable()) mq->launcher.join();
  std::free(mq->packets);
  delete mq;
  return HSA_STATUS_SUCCESS;
}
uint64_t hsa_queue_add_write_index_relaxed(const hsa_queue_t* q, uint64_t value) {
  return reinterpret_cast<MockQueue*>(q->id)->write_index.fetch_add(value);
}

hsa_status_t hsa_signal_create(hsa_signal_value_t initial, uint32_t, const hsa_agent_t*,
                               hsa_signal_t* s) {
  auto* m = new MockSignal();
  m->v.store(initial);
  s->handle = reinterpret_cast<uint64_t>(m);
  return HSA_STATUS_SUCCESS;
}
hsa_status_t hsa_signal_destroy(hsa_signal_t s) {
  delete sig(s);
  return HSA_STATUS_SUCCESS;
}
void hsa_signal_store_screlease(hsa_signal_t s, hsa_signal_value_t v) {
  MockSignal* m = sig(s);
  m->v.store(v, std::memory_order_release);
  if (MockQueue* mq = m->doorbell_of) {
    // the packet processor: one dispatch per queue in this model
    if (mq->launcher.joinable()) std::abort();
    mq->launcher = std::thread(run_dispatch, mq, (uint64_t)v);
  }
}
hsa_signal_value_t hsa_signal_wait_scacquire(hsa_signal_t s, hsa_signal_condition_t c,
                                             hsa_signal_value_t compare,
                                             uint64_t timeout_hint, hsa_wait_state_t) {
  // the hint in nanoseconds, at most 1 ms
  const auto until =
      Clock::now() + std::chrono::nanoseconds(timeout_hint < 1000000 ? timeout_hint : 1000000);
  for (;;) {
    const hsa_signal_value_t v = sig(s)->v.load(std::memory_order_acquire);
    bool met = false;
    switch (c) {
      case HSA_SIGNAL_CONDITION_EQ: met = v == compare; break;
      case HSA_SIGNAL_CONDITION_NE: met = v != compare; break;
      case HSA_SIGNAL_CONDITION_LT: met = v < compare; break;
      case HSA_SIGNAL_CONDITION_GTE: met = v >= compare; break;
    }
    if (met || Clock::now() >= until) return v;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}
