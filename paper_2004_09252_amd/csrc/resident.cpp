// Host side of the resident-key engine (include/memshield_resident.h; the
// kernel is in resident.hip).
//
// Producers: any number of host threads.  A submission takes the engine's
// mutex, checks that the ring slots of its positions are free (the kernel
// has completed their previous occupants), writes its descriptors into the
// pinned ring, and publishes the new count with a release store; the
// kernel's poller picks the count up over the link.  Completion: the kernel
// writes `position + 1` into the slot's completion word in pinned host
// memory after the pages; a ticket (first position, descriptor count) is
// done when every one of its positions has completed.
//
// Dispatch: the kernel never ends on its own while it has work, so it must
// not sit in a queue that other work shares (a shared in-order queue would
// hold everything behind it), and no stream of the HIP runtime may be made
// to wait for it.  It is therefore dispatched outside the HIP runtime: its
// code object (built separately and embedded in this library) is loaded
// with the HSA loader, and one AQL kernel-dispatch packet is written into an
// HSA queue created for this engine alone.  The packet's completion signal
// tells when the kernel has ended.
#include <hip/hip_runtime.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>
#include <sys/random.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "memshield_resident.h"
#include "ms_internal.h"
#include "ms_kernels.h"
#include "ms_resident_kernel.h"
#include "resident_shares.h"

static_assert(ms::kRkMaxKeys == MS_RESIDENT_MAX_KEYS, "key table size");

extern "C" const unsigned char ms_resident_code_object[];
extern "C" const size_t ms_resident_code_object_size;

struct ms_resident {
  ms_ctx* ctx = nullptr;
  int device = 0;
  ms_resident_config cfg{};
  uint32_t workers = 0;
  // HSA dispatch
  bool hsa_up = false;
  hsa_agent_t agent{};
  hsa_code_object_reader_t reader{};
  hsa_executable_t exe{};
  bool have_reader = false, have_exe = false;
  hsa_queue_t* queue = nullptr;
  hsa_signal_t done{};
  bool have_signal = false;
  void* kernarg = nullptr;        // pinned, the kernel's argument block
  hipStream_t aux = nullptr;      // key upload, debug reads
  ms::RkHostCtl* hctl = nullptr;  // pinned
  ms::RkDesc* ring = nullptr;     // pinned
  uint64_t* completed = nullptr;  // pinned, ring_depth words
  uint8_t* staging = nullptr;     // pinned, 32 bytes
  ms::RkDevCtl* dctl = nullptr;   // device
  uint32_t* key_buf = nullptr;    // device, n_keys x 8 words
  uint32_t n_keys = 1;
  bool launched = false;
  std::mutex mu;                  // producers
  // written under `mu` by producers; read without it by ms_resident_poll,
  // which must not contend with producers for the lock
  std::atomic<uint64_t> next_pos{0};
};

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint64_t kTicketCountBits = 24;

std::mutex g_reg_mu;
std::multimap<ms_ctx*, ms_resident*> g_engines;
// Every engine whose kernel was dispatched and not yet released, registered
// or not (a context's serving ring is not): what ms_internal_resident_live
// counts.
std::mutex g_live_mu;
std::set<ms_resident*> g_live;

bool hip_ok(hipError_t e) { return e == hipSuccess; }

template <class T>
T load_acq(const T* p) {
  return __atomic_load_n(p, __ATOMIC_ACQUIRE);
}
template <class T>
void store_rel(T* p, T v) {
  __atomic_store_n(p, v, __ATOMIC_RELEASE);
}

void wipe(void* p, size_t n) { explicit_bzero(p, n); }

// Wait for the dispatch's completion signal; false if `ms` elapsed first.
bool wait_kernel(ms_resident* r, uint64_t ms) {
  const auto deadline = Clock::now() + std::chrono::milliseconds(ms);
  // the wait's timeout hint is in system-timestamp ticks; a short one keeps
  // the deadline checked
  while (hsa_signal_wait_scacquire(r->done, HSA_SIGNAL_CONDITION_LT, 1,
                                   1000000, HSA_WAIT_STATE_BLOCKED) >= 1) {
    if (Clock::now() > deadline) return false;
  }
  return true;
}

// Stop the kernel, wait for it, free everything; false if the kernel did not
// end (its buffers are then kept).
bool release(ms_resident* r) {
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(r);
  }
  bool drained = true;
  if (r->launched) {
    store_rel(&r->hctl->stop, 1u);
    drained = wait_kernel(r, 60000);
    r->launched = false;
  }
  if (!drained) {
    // The kernel did not end (it reads `stop` on every poll, so this means
    // the device stopped making progress): keep every buffer it could touch.
    std::fprintf(stderr, "memshield: resident kernel did not stop; its "
                         "buffers are left allocated\n");
    return false;
  }
  if (r->queue) (void)hsa_queue_destroy(r->queue);
  if (r->have_signal) (void)hsa_signal_destroy(r->done);
  if (r->have_exe) (void)hsa_executable_destroy(r->exe);
  if (r->have_reader) (void)hsa_code_object_reader_destroy(r->reader);
  if (r->hsa_up) (void)hsa_shut_down();
  if (r->kernarg) (void)hipHostFree(r->kernarg);
  if (r->key_buf) {
    if (r->aux && hip_ok(hipMemsetAsync(r->key_buf, 0,
                                        (size_t)r->n_keys * MS_KEY_BYTES,
                                        r->aux)))
      (void)hipStreamSynchronize(r->aux);
    (void)hipFree(r->key_buf);
  }
  if (r->dctl) (void)hipFree(r->dctl);
  if (r->staging) {
    wipe(r->staging, MS_KEY_BYTES);
    (void)hipHostFree(r->staging);
  }
  if (r->ring) (void)hipHostFree(r->ring);
  if (r->completed) (void)hipHostFree(r->completed);
  if (r->hctl) (void)hipHostFree(r->hctl);
  if (r->aux) (void)hipStreamDestroy(r->aux);
  delete r;
  return true;
}

bool kernel_exited(ms_resident* r) {
  return load_acq(&r->hctl->exited) != 0;
}

struct AgentMatch {
  uint32_t domain, bus, dev;
  hsa_agent_t agent;
  bool found;
};

hsa_status_t match_agent(hsa_agent_t a, void* data) {
  auto* m = static_cast<AgentMatch*>(data);
  hsa_device_type_t type;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &type) !=
          HSA_STATUS_SUCCESS ||
      type != HSA_DEVICE_TYPE_GPU)
    return HSA_STATUS_SUCCESS;
  uint32_t bdf = 0, domain = 0;
  if (hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID,
                         &bdf) != HSA_STATUS_SUCCESS ||
      hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_DOMAIN,
                         &domain) != HSA_STATUS_SUCCESS)
    return HSA_STATUS_SUCCESS;
  if ((bdf >> 8) == m->bus && ((bdf >> 3) & 0x1fu) == m->dev &&
      domain == m->domain) {
    m->agent = a;
    m->found = true;
    return HSA_STATUS_INFO_BREAK;
  }
  return HSA_STATUS_SUCCESS;
}

const char* kernel_symbol(uint32_t cipher, int rounds) {
  const bool salsa = cipher == MS_CIPHER_SALSA;
  switch (rounds) {
    case 20: return salsa ? ms::kResidentSalsa20 : ms::kResidentKernel20;
    case 12: return salsa ? ms::kResidentSalsa12 : ms::kResidentKernel12;
    case 8: return salsa ? ms::kResidentSalsa8 : ms::kResidentKernel8;
  }
  return nullptr;
}

// Load the embedded code object on the context's GPU agent, create the
// engine's queue and completion signal, and write the dispatch packet.
ms_status dispatch(ms_resident* r, const ms::RkArgs& args, uint32_t cipher,
                   int rounds) {
  hipDeviceProp_t prop;
  if (!hip_ok(hipGetDeviceProperties(&prop, r->device))) return MS_EDEVICE;
  if (hsa_init() != HSA_STATUS_SUCCESS) return MS_EDEVICE;
  r->hsa_up = true;
  AgentMatch m{(uint32_t)prop.pciDomainID, (uint32_t)prop.pciBusID,
               (uint32_t)prop.pciDeviceID, {}, false};
  (void)hsa_iterate_agents(match_agent, &m);
  if (!m.found) return MS_EDEVICE;
  r->agent = m.agent;
  if (hsa_code_object_reader_create_from_memory(
          ms_resident_code_object, ms_resident_code_object_size,
          &r->reader) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  r->have_reader = true;
  if (hsa_executable_create_alt(HSA_PROFILE_FULL,
                                HSA_DEFAULT_FLOAT_ROUNDING_MODE_DEFAULT,
                                nullptr, &r->exe) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  r->have_exe = true;
  if (hsa_executable_load_agent_code_object(r->exe, r->agent, r->reader,
                                            nullptr, nullptr) !=
          HSA_STATUS_SUCCESS ||
      hsa_executable_freeze(r->exe, nullptr) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  const char* name = kernel_symbol(cipher, rounds);
  hsa_executable_symbol_t sym;
  uint64_t kernel_object = 0;
  uint32_t kernarg_size = 0, group_size = 0, private_size = 0;
  if (!name ||
      hsa_executable_get_symbol_by_name(r->exe, name, &r->agent, &sym) !=
          HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(
          sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT, &kernel_object) !=
          HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(
          sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE,
          &kernarg_size) != HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(
          sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE,
          &group_size) != HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(
          sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE,
          &private_size) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  // the key must never reach per-lane memory: refuse a kernel with scratch
  if (kernel_object == 0 || kernarg_size != sizeof(ms::RkArgs) ||
      private_size != 0)
    return MS_EDEVICE;
  if (!hip_ok(hipHostMalloc(&r->kernarg, 256, hipHostMallocDefault)))
    return MS_ENOMEM;
  std::memset(r->kernarg, 0, 256);
  std::memcpy(r->kernarg, &args, sizeof(args));
  uint32_t min_size = 0;
  if (hsa_agent_get_info(r->agent, HSA_AGENT_INFO_QUEUE_MIN_SIZE,
                         &min_size) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  const uint32_t qsize = min_size > 64 ? min_size : 64;
  if (hsa_queue_create(r->agent, qsize, HSA_QUEUE_TYPE_SINGLE, nullptr,
                       nullptr, UINT32_MAX, UINT32_MAX, &r->queue) !=
      HSA_STATUS_SUCCESS) {
    r->queue = nullptr;
    return MS_EDEVICE;
  }
  if (hsa_signal_create(1, 0, nullptr, &r->done) != HSA_STATUS_SUCCESS)
    return MS_EDEVICE;
  r->have_signal = true;
  const uint32_t waves = r->workers + 1;
  const uint32_t blocks = (waves + ms::kWavesPerBlock - 1) / ms::kWavesPerBlock;
  const uint64_t index = hsa_queue_add_write_index_relaxed(r->queue, 1);
  auto* pkt = static_cast<hsa_kernel_dispatch_packet_t*>(
                  r->queue->base_address) +
              (index & (r->queue->size - 1));
  std::memset(reinterpret_cast<uint8_t*>(pkt) + 4, 0, sizeof(*pkt) - 4);
  pkt->workgroup_size_x = (uint16_t)ms::kBlockThreads;
  pkt->workgroup_size_y = 1;
  pkt->workgroup_size_z = 1;
  pkt->grid_size_x = blocks * ms::kBlockThreads;
  pkt->grid_size_y = 1;
  pkt->grid_size_z = 1;
  pkt->private_segment_size = 0;
  pkt->group_segment_size = group_size;
  pkt->kernel_object = kernel_object;
  pkt->kernarg_address = r->kernarg;
  pkt->completion_signal = r->done;
  const uint16_t header =
      (HSA_PACKET_TYPE_KERNEL_DISPATCH << HSA_PACKET_HEADER_TYPE) |
      (1u << HSA_PACKET_HEADER_BARRIER) |
      (HSA_FENCE_SCOPE_SYSTEM << HSA_PACKET_HEADER_SCACQUIRE_FENCE_SCOPE) |
      (HSA_FENCE_SCOPE_SYSTEM << HSA_PACKET_HEADER_SCRELEASE_FENCE_SCOPE);
  const uint16_t setup = 1u << HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS;
  __atomic_store_n(reinterpret_cast<uint32_t*>(pkt),
                   (uint32_t)header | ((uint32_t)setup << 16),
                   __ATOMIC_RELEASE);
  hsa_signal_store_screlease(r->queue->doorbell_signal, (hsa_signal_value_t)index);
  r->launched = true;
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(r);
  }
  return MS_OK;
}

}  // namespace

void ms_internal_resident_stop_all(ms_ctx* c) {
  std::vector<ms_resident*> mine;
  {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto range = g_engines.equal_range(c);
    for (auto it = range.first; it != range.second; ++it)
      mine.push_back(it->second);
    g_engines.erase(c);
  }
  for (ms_resident* r : mine) release(r);
}

extern "C" {

void ms_resident_config_default(ms_resident_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->workers = 256;
  cfg->ring_depth = 4096;
  cfg->desc_pages = 16;
  cfg->idle_limit_ms = 10000;
}

}  // extern "C"

namespace {

// Start an engine with n_keys keys: from `key_bytes` (32 bytes, n_keys == 1),
// from the OS CSPRNG (both null, n_keys == 1), or copied device to device
// from the context's key table (`handles`).  With `table` (n_keys == 0) the
// engine holds no key: descriptors name rows of that device key table.  An
// engine started for the caller is registered with its context (stopped by
// ms_shutdown); one the context starts for itself (`registered` false) is
// the context's own to stop.
ms_status start_engine(ms_ctx* c, const ms_resident_config* cfg_in,
                       const uint8_t* key_bytes, const ms_key* handles,
                       uint32_t n_keys, ms_resident** out,
                       const uint32_t* table = nullptr,
                       uint32_t table_rows = 0, bool registered = true) {
  if (!c || !out) return MS_EINVAL;
  if (table ? (n_keys != 0 || table_rows == 0)
            : (n_keys == 0 || n_keys > ms::kRkMaxKeys))
    return MS_EINVAL;
  ms_status st = ms_internal_sticky(c);
  if (st) return st;
  ms_resident_config cfg;
  if (cfg_in) cfg = *cfg_in; else ms_resident_config_default(&cfg);
  const int rounds = (int)ms_internal_config(c).rounds;
  const uint32_t cipher = ms_internal_config(c).cipher;
  if (cfg.ring_depth < 16 || cfg.ring_depth > (1u << 20) ||
      (cfg.ring_depth & (cfg.ring_depth - 1)) || cfg.desc_pages == 0 ||
      cfg.desc_pages > 1024 || cfg.idle_limit_ms > 3600u * 1000u)
    return MS_EINVAL;
  if (!hip_ok(hipSetDevice(ms_internal_device(c)))) return MS_EDEVICE;
  // at most one workgroup per compute unit, so that every worker wave can be
  // resident at once next to other work (each must load the key)
  const uint32_t cap =
      (uint32_t)ms_internal_cu_count(c) * ms::kWavesPerBlock - 1;
  if (cfg.workers == 0 || cfg.workers > cap) return MS_EINVAL;
  int clock_khz = 0;
  if (!hip_ok(hipDeviceGetAttribute(&clock_khz,
                                    hipDeviceAttributeWallClockRate,
                                    ms_internal_device(c))) ||
      clock_khz <= 0)
    return MS_EDEVICE;

  ms_resident* r = new (std::nothrow) ms_resident();
  if (!r) return MS_ENOMEM;
  r->ctx = c;
  r->device = ms_internal_device(c);
  r->cfg = cfg;
  r->workers = cfg.workers;
  r->n_keys = n_keys;
  const size_t depth = cfg.ring_depth;
  const size_t key_bytes_total = (size_t)(table ? 1 : n_keys) * MS_KEY_BYTES;
  bool ok = hip_ok(hipStreamCreateWithFlags(&r->aux, hipStreamNonBlocking));
  if (!ok) {
    (void)hipGetLastError();
    release(r);
    return MS_EDEVICE;
  }
  // memory the running kernel and the host both read and write: coherent
  // (fine-grained) by request, whatever the runtime's default
  ok = hip_ok(hipHostMalloc(reinterpret_cast<void**>(&r->hctl),
                            sizeof(ms::RkHostCtl), hipHostMallocCoherent)) &&
       hip_ok(hipHostMalloc(reinterpret_cast<void**>(&r->ring),
                            depth * sizeof(ms::RkDesc),
                            hipHostMallocCoherent)) &&
       hip_ok(hipHostMalloc(reinterpret_cast<void**>(&r->completed),
                            depth * sizeof(uint64_t), hipHostMallocCoherent)) &&
       hip_ok(hipHostMalloc(reinterpret_cast<void**>(&r->staging),
                            MS_KEY_BYTES, hipHostMallocDefault)) &&
       hip_ok(hipMalloc(reinterpret_cast<void**>(&r->dctl),
                        sizeof(ms::RkDevCtl))) &&
       hip_ok(hipMalloc(reinterpret_cast<void**>(&r->key_buf),
                        key_bytes_total));
  if (!ok) {
    (void)hipGetLastError();
    release(r);
    return MS_ENOMEM;
  }
  std::memset(r->hctl, 0, sizeof(ms::RkHostCtl));
  std::memset(r->staging, 0, MS_KEY_BYTES);
  std::memset(r->ring, 0, depth * sizeof(ms::RkDesc));
  std::memset(r->completed, 0, depth * sizeof(uint64_t));
  hipError_t e = hipMemsetAsync(r->dctl, 0, sizeof(ms::RkDevCtl), r->aux);
  if (!hip_ok(e)) {
    release(r);
    return ms_internal_dev_err(c, e);
  }
  if (table) {
    // no key of its own: the device buffer stays zero
    e = hipMemsetAsync(r->key_buf, 0, key_bytes_total, r->aux);
    if (hip_ok(e)) e = hipStreamSynchronize(r->aux);
    if (!hip_ok(e)) {
      release(r);
      return ms_internal_dev_err(c, e);
    }
  } else if (handles) {
    // keys already on the device: copied from the context's key table, never
    // through host memory
    for (uint32_t i = 0; i < n_keys && !st; ++i)
      st = ms_internal_copy_key(c, handles[i], r->key_buf + (size_t)i * 8,
                                r->aux);
    if (st) {
      release(r);
      return st;
    }
  } else {
    // key: caller's bytes or the OS CSPRNG, into pinned staging, to the GPU,
    // then wiped from the staging buffer
    if (key_bytes) {
      std::memcpy(r->staging, key_bytes, MS_KEY_BYTES);
    } else {
      size_t got = 0;
      while (got < MS_KEY_BYTES) {
        const ssize_t n = getrandom(r->staging + got, MS_KEY_BYTES - got, 0);
        if (n < 0) {
          release(r);
          return MS_EDEVICE;
        }
        got += (size_t)n;
      }
    }
    e = hipMemcpyAsync(r->key_buf, r->staging, MS_KEY_BYTES,
                       hipMemcpyHostToDevice, r->aux);
    if (hip_ok(e)) e = hipStreamSynchronize(r->aux);
    wipe(r->staging, MS_KEY_BYTES);
    if (!hip_ok(e)) {
      release(r);
      return ms_internal_dev_err(c, e);
    }
  }
  ms::RkArgs a{};
  a.ring = r->ring;
  a.completed = r->completed;
  a.hctl = r->hctl;
  a.dctl = r->dctl;
  a.key_buf = r->key_buf;
  a.idle_ticks = (uint64_t)cfg.idle_limit_ms * (uint64_t)clock_khz;
  a.ring_mask = cfg.ring_depth - 1;
  a.n_workers = r->workers;
  a.max_pages = cfg.desc_pages;
  a.n_keys = n_keys;
  a.inv_step = ms::share_stride_inverse(r->workers);
  a.table_rows = table_rows;
  a.key_table = table;
  st = dispatch(r, a, cipher, rounds);
  if (st) {
    release(r);
    return st;
  }
  // wait for every worker to hold the keys (the kernel then wipes its copy)
  const auto deadline = Clock::now() + std::chrono::seconds(10);
  while (!load_acq(&r->hctl->ready)) {
    if (kernel_exited(r) || Clock::now() > deadline) {
      release(r);
      return MS_ETIMEDOUT;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (registered) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_engines.emplace(c, r);
  }
  *out = r;
  return MS_OK;
}

}  // namespace

ms_status ms_internal_ring_start(ms_ctx* c, const ms_resident_config* cfg,
                                 const uint32_t* key_table,
                                 uint32_t table_rows, ms_resident** out) {
  if (!key_table) return MS_EINVAL;
  return start_engine(c, cfg, nullptr, nullptr, 0, out, key_table,
                      table_rows, false);
}

ms_status ms_internal_ring_publish(ms_resident* r, uint32_t key_row,
                                   const void* src, void* dst,
                                   uint64_t n_pages, const ms_nonce& nonce,
                                   ms_ticket* ticket_out) {
  if (!r || n_pages == 0 || r->n_keys != 0) return MS_EINVAL;
  const uint64_t per = r->cfg.desc_pages;
  const uint64_t m = (n_pages + per - 1) / per;
  const uint64_t depth = r->cfg.ring_depth;
  if (m > depth) return MS_EINVAL;
  if (load_acq(&r->hctl->error)) return MS_EDEVICE;
  if (kernel_exited(r)) return MS_ECLOSED;
  const uint64_t s = reinterpret_cast<uint64_t>(src);
  const uint64_t d = reinterpret_cast<uint64_t>(dst);
  const uint64_t na = reinterpret_cast<uint64_t>(nonce.array);
  std::lock_guard<std::mutex> lk(r->mu);
  const uint64_t p0 = r->next_pos.load(std::memory_order_relaxed);
  for (uint64_t q = p0; q < p0 + m; ++q)
    if (q >= depth && load_acq(&r->completed[q & (depth - 1)]) < q - depth + 1)
      return MS_EAGAIN;
  for (uint64_t i = 0; i < m; ++i) {
    const uint64_t q = p0 + i;
    const uint64_t first = i * per;
    ms::RkDesc& x = r->ring[q & (depth - 1)];
    x.src = s + first * MS_PAGE_SIZE;
    x.dst = d + first * MS_PAGE_SIZE;
    if (nonce.kind == MS_NONCE_ARRAY) {
      x.nonce_base = na + first * MS_NONCE_BYTES;
      x.nonce_stride = 0;
      x.tag = 0;
      x.kind = 0;
    } else {
      x.nonce_base = nonce.base + first * nonce.stride;
      x.nonce_stride = nonce.stride;
      x.tag = nonce.tag;
      x.kind = 1;
    }
    x.n_pages = (uint32_t)(n_pages - first < per ? n_pages - first : per);
    x.key = key_row;
    x.seq = q;
  }
  store_rel(&r->hctl->published, p0 + m);
  r->next_pos.store(p0 + m, std::memory_order_release);
  *ticket_out = ((p0 + 1) << kTicketCountBits) | m;
  return MS_OK;
}

int ms_internal_ring_done(ms_resident* r, ms_ticket t) {
  const uint64_t depth = r->cfg.ring_depth;
  const uint64_t m = t & ((1ull << kTicketCountBits) - 1);
  const uint64_t p0 = (t >> kTicketCountBits) - 1;
  // last position first: it was published last and usually finishes last,
  // so a pending ticket costs one read of host memory the device writes
  // (a forward scan would reread a request's finished positions on every
  // poll, which under load made the scheduler's reaping grow with the
  // number of requests in flight)
  for (uint64_t q = p0 + m; q-- > p0;)
    if (load_acq(&r->completed[q & (depth - 1)]) < q + 1) return 0;
  return 1;
}

void ms_internal_ring_span(ms_ticket t, uint64_t* first, uint64_t* count) {
  *count = t & ((1ull << kTicketCountBits) - 1);
  *first = (t >> kTicketCountBits) - 1;
}

uint64_t ms_internal_ring_published(ms_resident* r) {
  return r->next_pos.load(std::memory_order_acquire);
}

uint64_t ms_internal_ring_advance(ms_resident* r, uint64_t from,
                                  uint64_t limit) {
  const uint64_t depth = r->cfg.ring_depth;
  while (from < limit && load_acq(&r->completed[from & (depth - 1)]) >= from + 1)
    ++from;
  return from;
}

uint32_t ms_internal_resident_live(int device) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  uint32_t n = 0;
  for (ms_resident* r : g_live)
    if (r->device == device && !kernel_exited(r)) ++n;
  return n;
}

bool ms_internal_ring_alive(ms_resident* r) {
  return r && r->launched && !kernel_exited(r) &&
         !load_acq(&r->hctl->error);
}

void ms_internal_ring_stop(ms_resident* r) {
  if (r) release(r);
}

extern "C" {

ms_status ms_resident_start(ms_ctx* c, const ms_resident_config* cfg,
                            const uint8_t* key, ms_resident** out) {
  return start_engine(c, cfg, key, nullptr, 1, out);
}

ms_status ms_resident_start_keys(ms_ctx* c, const ms_resident_config* cfg,
                                 const ms_key* keys, uint32_t n_keys,
                                 ms_resident** out) {
  if (!keys) return MS_EINVAL;
  return start_engine(c, cfg, nullptr, keys, n_keys, out);
}

ms_status ms_resident_submit(ms_resident* r, const void* src, void* dst,
                             uint64_t n_pages, const ms_nonce* nonce,
                             ms_ticket* ticket_out) {
  return ms_resident_submit_keyed(r, 0, src, dst, n_pages, nonce, ticket_out);
}

ms_status ms_resident_submit_keyed(ms_resident* r, uint32_t key_index,
                                   const void* src, void* dst,
                                   uint64_t n_pages, const ms_nonce* nonce,
                                   ms_ticket* ticket_out) {
  if (!r || !nonce || n_pages == 0 || key_index >= r->n_keys)
    return MS_EINVAL;
  if (nonce->kind != MS_NONCE_LINEAR && nonce->kind != MS_NONCE_ARRAY)
    return MS_EINVAL;
  if (n_pages > UINT64_MAX / MS_PAGE_SIZE) return MS_EINVAL;
  const uint64_t bytes = n_pages * MS_PAGE_SIZE;
  uint64_t s = 0, d = 0, na = 0;
  ms_status st = ms_internal_classify_any(r->ctx, src, bytes, 16, &s);
  if (st) return st;
  // in place: the same range, already classified
  if (dst == src)
    d = s;
  else if ((st = ms_internal_classify_any(r->ctx, dst, bytes, 16, &d)))
    return st;
  if (nonce->kind == MS_NONCE_ARRAY &&
      (st = ms_internal_classify_any(r->ctx, nonce->array,
                                     n_pages * MS_NONCE_BYTES, 4, &na)))
    return st;
  const uintptr_t a = reinterpret_cast<uintptr_t>(src);
  const uintptr_t b = reinterpret_cast<uintptr_t>(dst);
  if (a != b && a < b + bytes && b < a + bytes) return MS_EINVAL;
  const uint64_t per = r->cfg.desc_pages;
  const uint64_t m = (n_pages + per - 1) / per;
  const uint64_t depth = r->cfg.ring_depth;
  if (m > depth) return MS_EINVAL;
  if (load_acq(&r->hctl->error)) return MS_EDEVICE;
  if (kernel_exited(r)) return MS_ECLOSED;
  std::lock_guard<std::mutex> lk(r->mu);
  const uint64_t p0 = r->next_pos.load(std::memory_order_relaxed);
  // every slot must have completed its previous occupant (position - depth)
  for (uint64_t q = p0; q < p0 + m; ++q)
    if (q >= depth && load_acq(&r->completed[q & (depth - 1)]) < q - depth + 1)
      return MS_EAGAIN;
  for (uint64_t i = 0; i < m; ++i) {
    const uint64_t q = p0 + i;
    const uint64_t first = i * per;
    ms::RkDesc& x = r->ring[q & (depth - 1)];
    x.src = s + first * MS_PAGE_SIZE;
    x.dst = d + first * MS_PAGE_SIZE;
    if (nonce->kind == MS_NONCE_ARRAY) {
      x.nonce_base = na + first * MS_NONCE_BYTES;
      x.nonce_stride = 0;
      x.tag = 0;
      x.kind = 0;
    } else {
      x.nonce_base = nonce->base + first * nonce->stride;
      x.nonce_stride = nonce->stride;
      x.tag = nonce->tag;
      x.kind = 1;
    }
    x.n_pages = (uint32_t)(n_pages - first < per ? n_pages - first : per);
    x.key = key_index;
    x.seq = q;
  }
  store_rel(&r->hctl->published, p0 + m);
  r->next_pos.store(p0 + m, std::memory_order_release);
  if (ticket_out) *ticket_out = ((p0 + 1) << kTicketCountBits) | m;
  return MS_OK;
}

ms_status ms_resident_poll(ms_resident* r, const ms_ticket* tickets, size_t n,
                           int32_t* done_out, uint64_t timeout_ns) {
  if (!r || (n && (!tickets || !done_out))) return MS_EINVAL;
  const uint64_t depth = r->cfg.ring_depth;
  const uint64_t issued = r->next_pos.load(std::memory_order_acquire);
  for (size_t i = 0; i < n; ++i) {
    const uint64_t m = tickets[i] & ((1ull << kTicketCountBits) - 1);
    const uint64_t p1 = tickets[i] >> kTicketCountBits;
    if (m == 0 || p1 == 0 || p1 - 1 + m > issued) return MS_EINVAL;
  }
  const auto deadline = Clock::now() + std::chrono::nanoseconds(timeout_ns);
  uint64_t beat = 0;
  for (;;) {
    size_t pending = 0;
    const bool gone = kernel_exited(r);
    for (size_t i = 0; i < n; ++i) {
      const uint64_t m = tickets[i] & ((1ull << kTicketCountBits) - 1);
      const uint64_t p0 = (tickets[i] >> kTicketCountBits) - 1;
      bool done = true;
      for (uint64_t q = p0; q < p0 + m && done; ++q)
        done = load_acq(&r->completed[q & (depth - 1)]) >= q + 1;
      done_out[i] = done ? 1 : (gone ? MS_ECANCELED : 0);
      if (!done && !gone) ++pending;
    }
    if (pending == 0) return MS_OK;
    if (timeout_ns == 0 || Clock::now() >= deadline) return MS_ETIMEDOUT;
    // a waiting host counts as activity for the kernel's idle limit; spin
    // on host memory, giving the core away now and then
    if ((++beat & 1023) == 0) {
      __atomic_fetch_add(&r->hctl->heartbeat, 1, __ATOMIC_RELAXED);
      std::this_thread::yield();
    }
  }
}

int ms_resident_alive(ms_resident* r) {
  if (!r || !r->launched) return 0;
  return load_acq(&r->hctl->ready) && !kernel_exited(r) ? 1 : 0;
}

ms_status ms_resident_stop(ms_resident* r) {
  if (!r) return MS_OK;
  {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    for (auto it = g_engines.begin(); it != g_engines.end(); ++it)
      if (it->second == r) {
        g_engines.erase(it);
        break;
      }
  }
  return release(r) ? MS_OK : MS_ETIMEDOUT;
}

int ms_resident_debug_key_wiped(ms_resident* r) {
  if (!r) return -1;
  std::vector<uint32_t> dev((size_t)r->n_keys * 8, 1u);
  if (!hip_ok(hipMemcpyAsync(dev.data(), r->key_buf,
                             (size_t)r->n_keys * MS_KEY_BYTES,
                             hipMemcpyDeviceToHost, r->aux)) ||
      !hip_ok(hipStreamSynchronize(r->aux)))
    return -1;
  for (uint32_t w : dev)
    if (w) return 0;
  for (uint32_t i = 0; i < MS_KEY_BYTES; ++i)
    if (r->staging[i]) return 0;
  return 1;
}

}  // extern "C"
