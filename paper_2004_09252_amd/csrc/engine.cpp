// Host engine behind the C ABI of include/memshield.h.
//
// Responsibilities (MemShield, section 4.4 "GPU encryption" and section 3):
//   * the key store: a device key table, keys entering through a pinned
//     staging buffer that is wiped at once, never leaving the GPU again;
//   * argument validation, so that a bad size or pointer becomes an error
//     code instead of a GPU fault;
//   * plain launches (one run of pages, one key) and fused batched launches
//     (many requests, many keys, one persistent launch, replayed from a
//     captured hipGraph);
//   * the serving path: many host threads submit requests (the paper's
//     multiple-producer queue); one scheduler thread admits them into fused
//     launches as batch slots and the in-flight byte budget free up, so
//     batches overlap on the device, and marks tickets complete.
#include <hip/hip_runtime.h>
#include <sys/random.h>
#include <time.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "memshield.h"
#include "ms_internal.h"
#include "ms_kernels.h"
#include "tune_cache.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kMaxKeysLimit = 65536;
// Ring serving stage: requests up to this many pages go to the ring (one
// descriptor per page, so a request's pages run on as many workers at
// once); longer ones, which are bound by bandwidth rather than latency, go
// to the fused launches.
constexpr uint64_t kRingMaxPages = 1024;
// The ring stage's reaper runs at most this often while nothing is short,
// and reads the completion words of a request nobody has polled to
// completion only this long after its publication.
constexpr int kRingReapEveryUs = 10;
constexpr int kRingReapWordsAfterUs = 200;
static_assert(ms::kStaticBatchMaxRequests == MS_STATIC_BATCH_MAX_REQUESTS,
              "static batch limit");
static_assert(ms::kCipherChaCha == MS_CIPHER_CHACHA &&
                  ms::kCipherSalsa == MS_CIPHER_SALSA,
              "cipher ids");

inline bool hip_ok(hipError_t e) { return e == hipSuccess; }

// Wipe that the compiler may not drop.
void secure_zero(void* p, size_t n) {
  volatile uint8_t* v = static_cast<volatile uint8_t*>(p);
  for (size_t i = 0; i < n; ++i) v[i] = 0;
  std::atomic_signal_fence(std::memory_order_seq_cst);
}

bool ranges_overlap(uintptr_t a, uint64_t na, uintptr_t b, uint64_t nb) {
  return a < b + nb && b < a + na;
}

struct Tuning {
  uint32_t ppw = 4;
  uint32_t unroll = 1;
  uint32_t waves_per_cu = 32;
  double us = 0.0;
};

// One reusable batch buffer: pinned host descriptors, their device copy, a
// completion event and the graphs captured for this buffer.
struct BatchSlot {
  uint8_t* host = nullptr;    // pinned, DevBatchHdr + DevReq[capacity]
  uint8_t* dev = nullptr;     // device copy read by the kernel
  size_t capacity = 0;        // requests
  hipEvent_t done = nullptr;  // recorded after the launch that used it
  bool used = false;
  // graphs keyed by (unroll, ppw, grid)
  struct G {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr;
  };
  std::map<uint64_t, G> graphs;
};

// A request the scheduler owns.
struct Pending {
  ms_request req;
  uint32_t ticket_slot;
  bool prefetch;
};

// Demand requests waiting for the ring serving stage: one FIFO per client,
// served round robin.  A client with a backlog takes one turn per round, so
// a burst from one client delays another client's request by one request
// per waiting client, not by the whole burst; each client's own requests
// keep their order.
struct ClientQueues {
  std::unordered_map<uint32_t, std::deque<Pending>> fifo;
  std::deque<uint32_t> turn;  // clients with a non-empty FIFO, next first
  size_t n = 0;

  bool empty() const { return n == 0; }
  size_t size() const { return n; }
  void push(const Pending& p) {
    std::deque<Pending>& d = fifo[p.req.client];
    if (d.empty()) turn.push_back(p.req.client);
    d.push_back(p);
    ++n;
  }
  // The request whose turn it is (the queues must not be empty).
  const Pending& front() { return fifo[turn.front()].front(); }
  // Take that request; its client goes to the back of the round.
  void pop_front() {
    const uint32_t cl = turn.front();
    turn.pop_front();
    std::deque<Pending>& d = fifo[cl];
    d.pop_front();
    --n;
    if (d.empty())
      fifo.erase(cl);
    else
      turn.push_back(cl);
  }
  // Move one client's requests (all of them if `all`) into `out`.
  void take(uint32_t client, bool all, std::vector<Pending>* out) {
    for (auto it = fifo.begin(); it != fifo.end();) {
      if (all || it->first == client) {
        for (const Pending& p : it->second) out->push_back(p);
        n -= it->second.size();
        it = fifo.erase(it);
      } else {
        ++it;
      }
    }
    std::deque<uint32_t> keep;
    for (uint32_t cl : turn)
      if (fifo.count(cl)) keep.push_back(cl);
    turn.swap(keep);
  }
};

// A statistics counter that many submitting threads bump at once: one
// cache line per shard, each thread on a shard of its own (threads beyond
// the shard count share), summed when read.
class ShardedCounter {
 public:
  void add(uint64_t v) {
    shard_[shard_index()].v.fetch_add(v, std::memory_order_relaxed);
  }
  uint64_t load() const {
    uint64_t s = 0;
    for (const Shard& x : shard_) s += x.v.load(std::memory_order_relaxed);
    return s;
  }

 private:
  static constexpr unsigned kShards = 16;
  struct alignas(64) Shard {
    std::atomic<uint64_t> v{0};
  };
  static unsigned shard_index() {
    static std::atomic<unsigned> next{0};
    thread_local const unsigned mine = next.fetch_add(1) % kShards;
    return mine;
  }
  Shard shard_[kShards];
};

// A key slot's count of requests in flight, one cache line per slot:
// submitting threads of different clients and the reaper update
// neighbouring slots at once.
struct alignas(64) KeyRef : std::atomic<int64_t> {
  KeyRef() : std::atomic<int64_t>(0) {}
};

// One cache line per slot: neighbouring slots belong to different
// submitting threads and the reaper.
struct alignas(64) TicketSlot {
  std::atomic<uint32_t> gen{0};
  std::atomic<int32_t> state{0};  // 0 pending, 1 done, <0 ms_status
  // ring serving stage: the ring ticket once the request is published (0
  // before), so that ms_poll can read its completion words itself
  std::atomic<uint64_t> ring{0};
};

// What the reaper needs of a request published on the ring serving stage,
// kept at its first ring position modulo the ring depth.  The publisher
// stores `seq` (first position + 1) last, with release order, so a reaper
// that reads a matching `seq` sees the other fields.
struct RingMeta {
  std::atomic<uint64_t> seq{0};
  // first position + 1 once a poll has read all of the request's completion
  // words as done, so that the reaper need not read them again (a stale
  // poll of an earlier occupant writes its own position, which never
  // matches a later one)
  std::atomic<uint64_t> seen{0};
  Clock::time_point published{};
  uint32_t ticket_slot = 0;
  uint32_t key_slot = 0;
  uint64_t n_pages = 0;
};

// A reaped ring request on its way to completion.
struct RingDone {
  uint32_t ticket_slot;
  uint32_t key_slot;
  int32_t state;
};

struct InflightBatch {
  int slot;
  int stream;
  std::vector<uint32_t> tickets;
  std::vector<uint32_t> key_slots;
  uint64_t bytes;
};

}  // namespace

struct ms_ctx {
  int device = 0;
  ms_config cfg{};
  hipStream_t stream = nullptr;
  int cu_count = 0;
  std::string arch;
  uint32_t resident_plain_wpc[3] = {0, 0, 0};  // resident waves/CU, by unroll
  uint32_t resident_batch_wpc[3] = {0, 0, 0};  // by unroll

  // ---- key store ----
  std::mutex key_mu;
  uint32_t* d_keys = nullptr;       // max_keys x 8 words
  uint8_t* h_staging = nullptr;     // pinned, 32 bytes
  std::vector<uint32_t> key_gen;    // current generation per slot
  std::vector<uint8_t> key_live;
  std::unique_ptr<KeyRef[]> key_refs;  // submitted, unfinished

  // ---- batched launches from ms_process_batch ----
  std::mutex batch_mu;
  std::vector<BatchSlot> sync_slots;
  size_t sync_next = 0;

  // ---- ms_process_batch_static: no allocation after ms_init ----
  std::mutex static_mu;
  void* d_static = nullptr;        // this device's descriptor array
                                   // (address of `scratch`, page_cipher.hip)
  uint8_t* h_static = nullptr;     // pinned staging of the same size
  hipEvent_t static_done = nullptr;  // after the last launch that read it
  bool static_used = false;
  std::vector<uint32_t> static_slots;  // capacity kStaticBatchMaxRequests
  std::vector<std::pair<uintptr_t, uint64_t>> static_ranges;  // same

  // ---- tuning ----
  std::mutex tune_mu;
  std::map<uint32_t, Tuning> tuned;  // log2 bucket -> tuning
  bool forced = false;
  Tuning forced_tuning;

  // ---- serving ----
  std::vector<TicketSlot> tickets;
  std::mutex ticket_mu;
  std::vector<uint32_t> ticket_free;
  // the counters below that submitting threads and the reaper both update
  // each have a cache line of their own
  alignas(64) std::atomic<uint64_t> outstanding{0};

  std::mutex q_mu;  // submission queue (multiple producers)
  std::condition_variable q_cv;
  std::deque<Pending> demand_q;
  std::deque<Pending> prefetch_q;
  // ring serving stage: requests of at most kRingMaxPages pages
  ClientQueues ring_q;
  std::deque<Pending> ring_pf_q;
  // their sizes, written under q_mu and read without it, so that a
  // submission or a scheduler pass finds empty queues without the lock
  std::atomic<uint64_t> ring_q_n{0}, ring_pf_n{0};
  std::atomic<bool> stop{false};
  std::thread scheduler;

  // serve_slots, serve_free and inflight belong to whoever
  // holds sched_mu: the scheduler thread, or a submitting thread that finds
  // the lock free and launches its own batch at once
  std::mutex sched_mu;
  std::vector<BatchSlot> serve_slots;
  std::vector<hipStream_t> serve_streams;
  std::vector<int> serve_free;
  std::deque<InflightBatch> inflight;
  // page bytes admitted on either stage and not yet reaped (the admission
  // cap applies to it; reserve_admission takes from it atomically)
  alignas(64) std::atomic<uint64_t> inflight_bytes{0};

  // ring serving stage (serve_stage): a resident kernel on its own HSA
  // queue reads each request's pages from a descriptor ring in mapped
  // memory and writes a completion word per position.  Started at the first
  // submission and kept until ms_shutdown; `ring` is written once (under
  // sched_mu) and read without the lock by ms_poll.
  bool ring_mode = false;
  std::atomic<ms_resident*> ring{nullptr};
  bool ring_failed = false;                 // (sched_mu)
  // Requests are reaped in ring order: ring_reap_pos is the first position
  // of the oldest request not yet reaped, and ring_done_pos its copy for
  // ms_poll (every position below it is done).  Both move only forward, on
  // the thread that holds sched_mu.
  std::unique_ptr<RingMeta[]> ring_meta;    // ring_depth entries
  uint64_t ring_reap_pos = 0;               // (sched_mu)
  Clock::time_point ring_last_reap{};       // (sched_mu)
  std::atomic<uint64_t> ring_done_pos{0};
  std::vector<RingDone> ring_batch;         // the reaper's (sched_mu)
  alignas(64) std::atomic<uint64_t> ring_desc{0};  // ring positions held
  alignas(64) std::atomic<uint64_t> ring_reqs{0};  // published, not reaped
  uint32_t ring_depth = 1u << 16;
  uint32_t ring_workers = 0;

  std::atomic<int32_t> sticky_error{0};

  // ---- host-resident pages (host_pages.cpp) ----
  HostPath* host = nullptr;

  // ---- stats ----
  alignas(64) std::atomic<uint64_t> st_completed{0};  // the reaper's
  // bumped by every submission: sharded
  ShardedCounter st_submitted, st_pages, st_ring_direct;
  alignas(64) std::atomic<uint64_t> st_eagain{0},
      st_batches{0}, st_pf_issued{0}, st_pf_dropped{0},
      st_cancelled{0}, st_max_inflight{0},
      st_max_batch{0}, st_max_inflight_batches{0},
      st_ring_queued{0}, st_ring_max_queued{0}, st_ring_reap_ns{0};
};

namespace {

ms_status dev_err(ms_ctx* c, hipError_t e) {
  if (e == hipSuccess) return MS_OK;
  if (c) c->sticky_error.store(MS_EDEVICE);
  return MS_EDEVICE;
}

ms_status check_sticky(ms_ctx* c) {
  return c->sticky_error.load() ? MS_EDEVICE : MS_OK;
}

// A device range [p, p+bytes) must lie inside one device allocation.
// Allocations a call has already found valid: the requests of one call
// often share a buffer, and within a call the caller keeps every buffer
// alive (the ABI's ownership rule), so a later range inside one of them
// needs no runtime query.  Cleared by each call that uses it.
struct RangeMemo {
  static constexpr int kMax = 8;
  uintptr_t base[kMax];
  uint64_t size[kMax];
  int n = 0;
  bool covers(uintptr_t q, uint64_t bytes) const {
    for (int i = 0; i < n; ++i)
      if (q >= base[i] && bytes <= size[i] && q - base[i] <= size[i] - bytes)
        return true;
    return false;
  }
  void add(uintptr_t b, uint64_t sz) {
    base[n % kMax] = b;
    size[n % kMax] = sz;
    n = n < kMax ? n + 1 : kMax;
  }
};

ms_status check_device_range(ms_ctx* c, const void* p, uint64_t bytes,
                             uint64_t align, RangeMemo* memo = nullptr) {
  if (!p) return MS_EINVAL;
  if (reinterpret_cast<uintptr_t>(p) % align) return MS_EINVAL;
  if (!c->cfg.validate_pointers) return MS_OK;
  if (memo && memo->covers(reinterpret_cast<uintptr_t>(p), bytes))
    return MS_OK;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return MS_EINVAL;
  }
  if (attr.type != hipMemoryTypeDevice) return MS_EINVAL;
  if (attr.device != c->device) return MS_EINVAL;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) !=
      hipSuccess) {
    (void)hipGetLastError();
    return MS_EINVAL;
  }
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t q = reinterpret_cast<uintptr_t>(p);
  if (q < b || bytes > size || q - b > size - bytes) return MS_EINVAL;
  if (memo) memo->add(b, size);
  return MS_OK;
}

bool resolve_key(ms_ctx* c, ms_key k, uint32_t* slot) {
  if (k == 0) return false;
  const uint32_t s = (uint32_t)(k & 0xffffffffu);
  const uint32_t g = (uint32_t)(k >> 32);
  if (s == 0 || s > c->cfg.max_keys) return false;
  std::lock_guard<std::mutex> lk(c->key_mu);
  if (!c->key_live[s - 1] || c->key_gen[s - 1] != g) return false;
  *slot = s - 1;
  return true;
}

// A synchronous call pins the key-table rows it uses from its handle check
// until its launches are on their streams: under the key lock it re-checks
// each handle and takes a reference.  ms_key_destroy then either sees the
// reference (MS_EBUSY) or runs after the launches were enqueued, so that its
// device synchronization covers them; a destroyed and reused row can never
// reach a launch that resolved the old handle.
ms_status pin_keys(ms_ctx* c, const ms_key* handles, size_t stride_bytes,
                   const uint32_t* slots, size_t n) {
  std::lock_guard<std::mutex> lk(c->key_mu);
  const uint8_t* h = reinterpret_cast<const uint8_t*>(handles);
  for (size_t i = 0; i < n; ++i) {
    ms_key k;
    std::memcpy(&k, h + i * stride_bytes, sizeof(k));
    if (!c->key_live[slots[i]] || c->key_gen[slots[i]] != (uint32_t)(k >> 32))
      return MS_ENOKEY;
  }
  for (size_t i = 0; i < n; ++i) c->key_refs[slots[i]].fetch_add(1);
  return MS_OK;
}

void unpin_keys(ms_ctx* c, const uint32_t* slots, size_t n) {
  for (size_t i = 0; i < n; ++i) c->key_refs[slots[i]].fetch_sub(1);
}

// Releases pinned rows when the call returns, on every path.
struct KeyPins {
  ms_ctx* c;
  const uint32_t* slots;
  size_t n = 0;
  ~KeyPins() {
    if (n) unpin_keys(c, slots, n);
  }
};

ms_status check_nonce(ms_ctx* c, const ms_nonce* n, uint64_t n_pages,
                      RangeMemo* memo = nullptr) {
  if (!n) return MS_EINVAL;
  if (n->kind == MS_NONCE_ARRAY) {
    if (n_pages > (UINT64_MAX / 12)) return MS_EINVAL;
    return check_device_range(c, n->array, n_pages * 12u, 4, memo);
  }
  if (n->kind == MS_NONCE_LINEAR) return MS_OK;
  return MS_EINVAL;
}

// Validate one request (pages, pointers, overlap, key, nonce).  With
// `resolve` false the key handle is only decoded into its slot: the caller
// checks it under the key lock itself.
ms_status check_request(ms_ctx* c, const ms_request& r, uint32_t* slot,
                        bool allow_empty, bool resolve = true,
                        RangeMemo* memo = nullptr) {
  if (r.priority != 0 || r.flags != 0) return MS_EINVAL;
  if (r.op != MS_ENCRYPT && r.op != MS_DECRYPT) return MS_EINVAL;
  if (r.n_pages == 0) {
    if (!allow_empty) return MS_EINVAL;
  } else {
    if (r.n_pages > (UINT64_MAX / MS_PAGE_SIZE)) return MS_EINVAL;
    const uint64_t bytes = r.n_pages * MS_PAGE_SIZE;
    ms_status st = check_device_range(c, r.src, bytes, 16, memo);
    if (st) return st;
    // in place: the same range, already checked
    if (r.dst != r.src &&
        (st = check_device_range(c, r.dst, bytes, 16, memo)))
      return st;
    const uintptr_t s = reinterpret_cast<uintptr_t>(r.src);
    const uintptr_t d = reinterpret_cast<uintptr_t>(r.dst);
    if (s != d && ranges_overlap(s, bytes, d, bytes)) return MS_EINVAL;
    st = check_nonce(c, &r.nonce, r.n_pages, memo);
    if (st) return st;
  }
  if (!resolve) {
    const uint32_t ks = (uint32_t)(r.key & 0xffffffffu);
    if (ks == 0 || ks > c->cfg.max_keys) return MS_ENOKEY;
    *slot = ks - 1;
    return MS_OK;
  }
  if (!resolve_key(c, r.key, slot)) return MS_ENOKEY;
  return MS_OK;
}

uint32_t bucket_of(uint64_t n_pages) {
  uint32_t b = 0;
  while ((1ull << b) < n_pages && b < 63) ++b;
  return b;
}

Tuning default_tuning(uint64_t n_pages) {
  Tuning t;
  t.unroll = 2;
  t.ppw = n_pages >= (1u << 16) ? 8 : (n_pages >= 4096 ? 4 : 2);
  t.waves_per_cu = 32;  // capped at the kernel's residency when launched
  return t;
}

Tuning tuning_for(ms_ctx* c, uint64_t n_pages) {
  std::lock_guard<std::mutex> lk(c->tune_mu);
  if (c->forced) return c->forced_tuning;
  auto it = c->tuned.find(bucket_of(n_pages));
  if (it != c->tuned.end()) return it->second;
  return default_tuning(n_pages);
}

// Plain launches: persistent waves, as many as fit on the chip at once.  At
// full residency the unroll-1 kernel (51-56 VGPRs, 8 waves per SIMD) hides
// memory latency across its waves and measured ~1% faster than the
// unroll-2 kernel (65-71 VGPRs, 7 waves per SIMD), whose waves keep their
// next page's loads in flight during the current page's rounds; 8 waves
// per SIMD also split 2^18 pages evenly (32 per wave).  A launch capped to
// few waves (pages in host memory, bound by the link) keeps unroll 2, where
// each wave's own overlap is what hides the latency.
// Wave slots per compute unit that resident kernels running on the device
// hold (one wave per SIMD each): a grid sized for an idle device would
// leave its last workgroups to start only after the first ones finish.
uint32_t resident_busy_wpc(ms_ctx* c) {
  return ms::kWavesPerBlock * ms_internal_resident_live(c->device);
}

Tuning plain_tuning(ms_ctx* c, bool capped) {
  Tuning t;
  t.ppw = 1;
  t.unroll = capped ? 2 : 1;
  uint32_t wpc = c->resident_plain_wpc[t.unroll];
  if (!wpc) wpc = 28;
  const uint32_t busy = resident_busy_wpc(c);
  t.waves_per_cu = wpc > busy + ms::kWavesPerBlock ? wpc - busy
                                                   : ms::kWavesPerBlock;
  return t;
}

uint32_t grid_blocks_for(ms_ctx* c, const Tuning& t, uint64_t total_pages) {
  const uint64_t items = (total_pages + t.ppw - 1) / t.ppw;
  uint32_t wpc = t.waves_per_cu;
  uint32_t res = c->resident_batch_wpc[t.unroll == 2 ? 2 : 1];
  // resident kernels on the device hold some of the slots
  const uint32_t busy = resident_busy_wpc(c);
  if (res) res = res > busy + ms::kWavesPerBlock ? res - busy
                                                 : ms::kWavesPerBlock;
  if (res && wpc > res) wpc = res;  // waves beyond residency start late
  const uint64_t max_waves = (uint64_t)c->cu_count * wpc;
  uint64_t waves = std::min<uint64_t>(std::max<uint64_t>(items, 1), max_waves);
  uint64_t blocks = (waves + ms::kWavesPerBlock - 1) / ms::kWavesPerBlock;
  return (uint32_t)std::max<uint64_t>(blocks, 1);
}

ms_status alloc_slot(BatchSlot& s, size_t capacity) {
  const size_t bytes =
      sizeof(ms::DevBatchHdr) + capacity * sizeof(ms::DevReq);
  // fine-grained: the descriptor copy kernel reads it over the link
  if (!hip_ok(hipHostMalloc(reinterpret_cast<void**>(&s.host), bytes,
                            hipHostMallocCoherent)))
    return MS_ENOMEM;
  if (!hip_ok(hipMalloc(reinterpret_cast<void**>(&s.dev), bytes)))
    return MS_ENOMEM;
  if (!hip_ok(hipEventCreateWithFlags(&s.done, hipEventDisableTiming)))
    return MS_EDEVICE;
  std::memset(s.host, 0, bytes);
  s.capacity = capacity;
  return MS_OK;
}

void free_slot(BatchSlot& s) {
  for (auto& kv : s.graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  s.graphs.clear();
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.dev) (void)hipFree(s.dev);
  if (s.host) (void)hipHostFree(s.host);
  s = BatchSlot();
}

// Lay the requests out as a batch header and request records in `host`
// (pinned).  Empty requests are skipped.  Returns the number of bytes to
// copy (0 when there is no work).  req(i) returns request i.
template <class Req>
size_t fill_descriptors(uint8_t* host, Req req, const uint32_t* key_slots,
                        size_t n, uint64_t* total_out) {
  auto* hdr = reinterpret_cast<ms::DevBatchHdr*>(host);
  auto* dr = reinterpret_cast<ms::DevReq*>(hdr + 1);
  uint64_t total = 0;
  uint32_t m = 0;
  for (size_t i = 0; i < n; ++i) {
    const ms_request& r = req(i);
    if (r.n_pages == 0) continue;
    ms::DevReq& d = dr[m++];
    d.src = reinterpret_cast<uint64_t>(r.src);
    d.dst = reinterpret_cast<uint64_t>(r.dst);
    if (r.nonce.kind == MS_NONCE_ARRAY) {
      d.kind = ms::kNonceArray;
      d.nonce = reinterpret_cast<uint64_t>(r.nonce.array);
      d.stride = 0;
      d.tag = 0;
    } else {
      d.kind = ms::kNonceLinear;
      d.nonce = r.nonce.base;
      d.stride = r.nonce.stride;
      d.tag = r.nonce.tag;
    }
    d.page_begin = total;
    total += r.n_pages;
    d.page_end = total;
    d.key_slot = key_slots[i];
    d.pad = 0;
  }
  hdr->total_pages = total;
  hdr->n_req = m;
  *total_out = total;
  if (m == 0) return 0;
  return sizeof(ms::DevBatchHdr) + (size_t)m * sizeof(ms::DevReq);
}

size_t fill_slot(BatchSlot& s, const ms_request* const* reqs,
                 const uint32_t* key_slots, size_t n, uint64_t* total_out) {
  return fill_descriptors(
      s.host, [reqs](size_t i) -> const ms_request& { return *reqs[i]; },
      key_slots, n, total_out);
}

// Destinations of a batch must not overlap each other, nor any source other
// than their own request's (in place is allowed).  `d` is working storage
// (cleared here; no allocation while its capacity covers n).
ms_status check_batch_ranges(const ms_request* reqs, size_t n,
                             std::vector<std::pair<uintptr_t, uint64_t>>& d) {
  d.clear();
  for (size_t i = 0; i < n; ++i)
    if (reqs[i].n_pages)
      d.emplace_back(reinterpret_cast<uintptr_t>(reqs[i].dst),
                     reqs[i].n_pages * MS_PAGE_SIZE);
  std::sort(d.begin(), d.end());
  for (size_t i = 1; i < d.size(); ++i)
    if (d[i - 1].first + d[i - 1].second > d[i].first) return MS_EINVAL;
  for (size_t i = 0; i < n; ++i) {
    if (!reqs[i].n_pages) continue;
    const uintptr_t s = reinterpret_cast<uintptr_t>(reqs[i].src);
    const uintptr_t own = reinterpret_cast<uintptr_t>(reqs[i].dst);
    const uint64_t nb = reqs[i].n_pages * MS_PAGE_SIZE;
    // destinations are disjoint and sorted, so their ends are sorted too:
    // walk back from the last one that starts before this source ends
    auto it = std::lower_bound(d.begin(), d.end(),
                               std::make_pair(s + nb, (uint64_t)0));
    while (it != d.begin()) {
      --it;
      if (it->first + it->second <= s) break;
      if (it->first == own && own == s) continue;  // in place
      return MS_EINVAL;
    }
  }
  return MS_OK;
}

// Kernel-node parameters of the descriptor copy of `bytes` out of slot s;
// `a` holds the argument values that *p points to.
struct CopyNodeArgs {
  void* dev;
  const void* host;
  uint32_t n16;
  void* args[3];
};

void copy_node_params(BatchSlot& s, size_t bytes, hipKernelNodeParams* p,
                      CopyNodeArgs* a) {
  a->dev = s.dev;
  a->host = s.host;
  a->n16 = (uint32_t)(bytes / 16);
  a->args[0] = &a->dev;
  a->args[1] = &a->host;
  a->args[2] = &a->n16;
  void** args = a->args;
  std::memset(p, 0, sizeof(*p));
  p->func = const_cast<void*>(ms::desc_copy_fn());
  p->gridDim = dim3(ms::desc_copy_blocks(bytes));
  p->blockDim = dim3(ms::kBlockThreads);
  p->sharedMemBytes = 0;
  p->kernelParams = args;
  p->extra = nullptr;
}

// Capture [copy descriptors H2D] -> [fused kernel] for this slot and tiling.
ms_status get_graph(ms_ctx* c, BatchSlot& s, const Tuning& t, uint32_t grid,
                    BatchSlot::G** out) {
  const uint64_t key = ((uint64_t)t.unroll << 56) ^ ((uint64_t)t.ppw << 32) ^
                       (uint64_t)grid;
  auto it = s.graphs.find(key);
  if (it != s.graphs.end()) {
    *out = &it->second;
    return MS_OK;
  }
  BatchSlot::G g;
  if (!hip_ok(hipGraphCreate(&g.graph, 0))) return MS_EDEVICE;
  // the descriptor copy is a kernel node (set to the batch's size at each
  // replay), so both nodes run on the launching queue
  const size_t full =
      sizeof(ms::DevBatchHdr) + s.capacity * sizeof(ms::DevReq);
  hipKernelNodeParams cp;
  CopyNodeArgs ca;
  copy_node_params(s, full, &cp, &ca);
  hipError_t e = hipGraphAddKernelNode(&g.copy, g.graph, nullptr, 0, &cp);
  if (!hip_ok(e)) {
    (void)hipGraphDestroy(g.graph);
    return dev_err(c, e);
  }
  const ms::DevBatchHdr* hdr = reinterpret_cast<const ms::DevBatchHdr*>(s.dev);
  const uint32_t* keys = c->d_keys;
  uint32_t ppw = t.ppw;
  void* args[] = {(void*)&hdr, (void*)&keys, (void*)&ppw};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = const_cast<void*>(ms::batch_kernel_fn(t.unroll, c->cfg.cipher, (int)c->cfg.rounds));
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(ms::kBlockThreads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  hipGraphNode_t kn;
  e = hipGraphAddKernelNode(&kn, g.graph, &g.copy, 1, &kp);
  if (!hip_ok(e)) {
    (void)hipGraphDestroy(g.graph);
    return dev_err(c, e);
  }
  e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (!hip_ok(e)) {
    (void)hipGraphDestroy(g.graph);
    return dev_err(c, e);
  }
  auto ins = s.graphs.emplace(key, g);
  *out = &ins.first->second;
  return MS_OK;
}

// Issue a filled slot on `stream`: graph replay, or direct launches (the
// records in the kernel arguments for a batch of at most kInlineBatchMax
// requests, else a descriptor copy and the batch kernel).
ms_status issue_slot(ms_ctx* c, BatchSlot& s, size_t copy_bytes,
                     uint64_t total, hipStream_t stream, bool use_graph) {
  const Tuning t = tuning_for(c, total);
  const uint32_t grid = grid_blocks_for(c, t, total);
  hipError_t e;
  if (use_graph) {
    BatchSlot::G* g = nullptr;
    ms_status st = get_graph(c, s, t, grid, &g);
    if (st) return st;
    hipKernelNodeParams cp;
    CopyNodeArgs ca;
    copy_node_params(s, copy_bytes, &cp, &ca);
    e = hipGraphExecKernelNodeSetParams(g->exec, g->copy, &cp);
    if (!hip_ok(e)) return dev_err(c, e);
    e = hipGraphLaunch(g->exec, stream);
    if (!hip_ok(e)) return dev_err(c, e);
  } else if (copy_bytes <= sizeof(ms::InlineBatch)) {
    // a small batch: its records go in the kernel arguments, so no
    // descriptor copy runs (and waits for this thread's second launch call)
    // ahead of the batch kernel
    ms::InlineBatch ib;
    std::memcpy(&ib, s.host, copy_bytes);
    e = ms::launch_batch_inline(ib, c->d_keys, t.ppw, t.unroll, grid,
                                c->cfg.cipher, (int)c->cfg.rounds, stream);
    if (!hip_ok(e)) return dev_err(c, e);
  } else {
    e = ms::launch_desc_copy(s.dev, s.host, copy_bytes, stream);
    if (!hip_ok(e)) return dev_err(c, e);
    e = ms::launch_batch(reinterpret_cast<const ms::DevBatchHdr*>(s.dev),
                         c->d_keys, t.ppw, t.unroll, grid, c->cfg.cipher,
                         (int)c->cfg.rounds,
                         stream);
    if (!hip_ok(e)) return dev_err(c, e);
  }
  e = hipEventRecord(s.done, stream);
  if (!hip_ok(e)) return dev_err(c, e);
  s.used = true;
  return MS_OK;
}

// ------------------------------------------------------------ scheduler ---

void finish_batch(ms_ctx* c, InflightBatch& b, int32_t state) {
  for (uint32_t ks : b.key_slots) c->key_refs[ks].fetch_sub(1);
  {
    std::lock_guard<std::mutex> lk(c->ticket_mu);
    for (uint32_t t : b.tickets) {
      c->tickets[t].state.store(state, std::memory_order_release);
      c->ticket_free.push_back(t);
    }
  }
  c->outstanding.fetch_sub(b.tickets.size());
  c->st_completed.fetch_add(b.tickets.size());
  c->inflight_bytes.fetch_sub(b.bytes);
  c->serve_free.push_back(b.slot);
}

// Take `bytes` of the admission cap and `positions` ring positions, both or
// neither.  Lock-free: submitting threads and the scheduler reserve at once.
bool reserve_admission(ms_ctx* c, uint64_t bytes, uint64_t positions) {
  const uint64_t cap = c->cfg.admission_cap_bytes;
  uint64_t b = c->inflight_bytes.load(std::memory_order_relaxed);
  do {
    if (b + bytes > cap) return false;
  } while (!c->inflight_bytes.compare_exchange_weak(b, b + bytes));
  if (positions) {
    uint64_t d = c->ring_desc.load(std::memory_order_relaxed);
    do {
      if (d + positions > c->ring_depth) {
        c->inflight_bytes.fetch_sub(bytes);
        return false;
      }
    } while (!c->ring_desc.compare_exchange_weak(d, d + positions));
  }
  const uint64_t now = b + bytes;
  uint64_t hi = c->st_max_inflight.load(std::memory_order_relaxed);
  while (now > hi && !c->st_max_inflight.compare_exchange_weak(hi, now)) {
  }
  return true;
}

void complete_ticket_now(ms_ctx* c, uint32_t t, int32_t state,
                         uint32_t key_slot) {
  c->key_refs[key_slot].fetch_sub(1);
  {
    std::lock_guard<std::mutex> lk(c->ticket_mu);
    c->tickets[t].state.store(state, std::memory_order_release);
    c->ticket_free.push_back(t);
  }
  c->outstanding.fetch_sub(1);
}

// Poll in-flight batches; returns true when any completed.
bool reap(ms_ctx* c) {
  bool any = false;
  for (auto it = c->inflight.begin(); it != c->inflight.end();) {
    hipError_t q = hipEventQuery(c->serve_slots[it->slot].done);
    if (q == hipErrorNotReady) {
      ++it;
      continue;
    }
    int32_t state = 1;
    if (q != hipSuccess) {
      c->sticky_error.store(MS_EDEVICE);
      state = MS_EDEVICE;
    }
    finish_batch(c, *it, state);
    it = c->inflight.erase(it);
    any = true;
  }
  return any;
}

// Form and launch one batch from the queues; returns false if nothing
// could be launched.
bool tuning_forced(ms_ctx* c) {
  std::lock_guard<std::mutex> lk(c->tune_mu);
  return c->forced;
}

bool launch_one(ms_ctx* c) {
  if (c->serve_free.empty()) return false;
  std::vector<Pending> take;
  const uint64_t cap = c->cfg.admission_cap_bytes;
  uint64_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(c->q_mu);
    const size_t maxn = c->cfg.max_batch_requests;
    while (!c->demand_q.empty() && take.size() < maxn) {
      const uint64_t b = c->demand_q.front().req.n_pages * MS_PAGE_SIZE;
      if (!reserve_admission(c, b, 0)) break;
      bytes += b;
      take.push_back(c->demand_q.front());
      c->demand_q.pop_front();
    }
    // prefetch hints only ride along when no demand request is waiting
    if (c->demand_q.empty()) {
      while (!c->prefetch_q.empty() && take.size() < maxn) {
        const uint64_t b = c->prefetch_q.front().req.n_pages * MS_PAGE_SIZE;
        if (!reserve_admission(c, b, 0)) break;
        bytes += b;
        take.push_back(c->prefetch_q.front());
        c->prefetch_q.pop_front();
      }
    }
  }
  (void)cap;
  if (take.empty()) return false;
  const int slot = c->serve_free.back();
  c->serve_free.pop_back();
  const int stream_i = slot % (int)c->serve_streams.size();
  BatchSlot& s = c->serve_slots[slot];
  std::vector<const ms_request*> rp(take.size());
  std::vector<uint32_t> ks(take.size());
  InflightBatch b;
  b.slot = slot;
  b.stream = stream_i;
  b.bytes = bytes;
  uint64_t n_pf = 0;
  for (size_t i = 0; i < take.size(); ++i) {
    rp[i] = &take[i].req;
    // the key slot was resolved and referenced at submit time
    ks[i] = (uint32_t)(take[i].req.key & 0xffffffffu) - 1;
    b.tickets.push_back(take[i].ticket_slot);
    b.key_slots.push_back(ks[i]);
    n_pf += take[i].prefetch ? 1 : 0;
  }
  uint64_t total = 0;
  const size_t copy = fill_slot(s, rp.data(), ks.data(), take.size(), &total);
  if (take.size() > c->st_max_batch.load()) c->st_max_batch.store(take.size());
  c->st_batches.fetch_add(1);
  c->st_pages.add(total);
  c->st_pf_issued.fetch_add(n_pf);
  ms_status st = MS_OK;
  hipStream_t strm = c->serve_streams[stream_i];
  if (copy && take.size() == 1 && !tuning_forced(c)) {
    // a batch of one request needs no descriptors: plain launch (unless a
    // caller has forced the fused launch's tuning for every batch)
    const ms_request& r = take[0].req;
    ms::PlainArgs a;
    a.keys = c->d_keys;
    a.src = static_cast<const uint8_t*>(r.src);
    a.dst = static_cast<uint8_t*>(r.dst);
    a.nonce_array = reinterpret_cast<const uint32_t*>(r.nonce.array);
    a.nonce_base = r.nonce.base;
    a.nonce_stride = r.nonce.stride;
    a.first_page = 0;
    a.n_pages = r.n_pages;
    a.key_slot = ks[0];
    a.nonce_tag = r.nonce.tag;
    const Tuning t = plain_tuning(c, false);
    hipError_t e = ms::launch_plain(
        a, r.nonce.kind == MS_NONCE_ARRAY ? ms::kNonceArray : ms::kNonceLinear,
        c->cfg.cipher, (int)c->cfg.rounds,
        (uint32_t)c->cu_count * t.waves_per_cu, t.unroll,
        strm);
    if (hip_ok(e)) e = hipEventRecord(s.done, strm);
    if (!hip_ok(e)) st = dev_err(c, e);
    s.used = true;
  } else if (copy) {
    st = issue_slot(c, s, copy, total, strm, false);
  } else if (!hip_ok(hipEventRecord(s.done, strm))) {
    st = MS_EDEVICE;
  }
  if (st != MS_OK) {
    finish_batch(c, b, st);
    return true;
  }
  c->inflight.push_back(std::move(b));
  if (c->inflight.size() > c->st_max_inflight_batches.load())
    c->st_max_inflight_batches.store(c->inflight.size());
  return true;
}

// ------------------------------------------------------ ring serving ---

// Start the ring at the first use (caller holds sched_mu).
ms_status ensure_ring(ms_ctx* c) {
  if (c->ring.load(std::memory_order_relaxed)) return MS_OK;
  if (c->ring_failed) return MS_EDEVICE;
  ms_resident_config rc;
  ms_resident_config_default(&rc);
  rc.workers = c->ring_workers;
  rc.ring_depth = c->ring_depth;
  rc.desc_pages = 1;
  rc.idle_limit_ms = 0;  // runs until ms_shutdown
  ms_resident* r = nullptr;
  const ms_status st =
      ms_internal_ring_start(c, &rc, c->d_keys, c->cfg.max_keys, &r);
  if (st) {
    c->ring_failed = true;
    return st;
  }
  c->ring.store(r, std::memory_order_release);
  return MS_OK;
}

// Publish one queued request whose admission bytes and ring positions are
// already reserved; on failure its ticket completes with the error.  Any
// thread may call it (the ring has its own lock; the reaper finds the
// request through its ring position).
void publish_reserved(ms_ctx* c, ms_resident* r, const Pending& p) {
  const uint32_t ks = (uint32_t)(p.req.key & 0xffffffffu) - 1;
  const uint64_t bytes = p.req.n_pages * MS_PAGE_SIZE;
  ms_ticket rt = 0;
  const ms_status st = ms_internal_ring_publish(
      r, ks, p.req.src, p.req.dst, p.req.n_pages, p.req.nonce, &rt);
  if (st) {
    // (MS_EAGAIN cannot happen: positions are counted until reaped)
    c->sticky_error.store(MS_EDEVICE);
    c->inflight_bytes.fetch_sub(bytes);
    c->ring_desc.fetch_sub(p.req.n_pages);
    complete_ticket_now(c, p.ticket_slot, st == MS_EAGAIN ? MS_EDEVICE : st,
                        ks);
    return;
  }
  uint64_t first = 0, count = 0;
  ms_internal_ring_span(rt, &first, &count);
  c->ring_reqs.fetch_add(1);
  c->tickets[p.ticket_slot].ring.store(rt, std::memory_order_release);
  RingMeta& m = c->ring_meta[first & (c->ring_depth - 1)];
  m.ticket_slot = p.ticket_slot;
  m.key_slot = ks;
  m.n_pages = count;
  m.published = Clock::now();
  m.seq.store(first + 1, std::memory_order_release);
  c->st_pages.add(p.req.n_pages);
  if (p.prefetch) c->st_pf_issued.fetch_add(1);
}

// Complete finished ring requests (caller holds sched_mu); true when any
// was.  Requests are taken in ring order from the oldest, and the walk stops
// at the first that is not finished (or whose publisher has not yet
// recorded it).  A request a poll has already seen finished costs no read of
// host memory.  Any other is left to its client's polls for
// kRingReapWordsAfterUs after its publication, unless ring positions,
// tickets or admission run short; after that the reaper checks its
// completion words itself, last position first (the unfinished head costs
// one read).  So in the usual case, where clients poll, each completion
// word is read by one thread only.  What the finished requests hold
// (tickets, admission bytes, ring positions) is released together, under
// one lock, and every position before the walk's end is then known
// complete (the prefix ms_poll reads first).
bool ring_reap(ms_ctx* c) {
  ms_resident* r = c->ring.load(std::memory_order_acquire);
  if (!r || c->ring_reqs.load(std::memory_order_acquire) == 0) return false;
  // Clients see completion in the completion words, not through the
  // reaper, so while nothing is short (no request waits for positions, the
  // ring and the tickets are less than half used) a pass runs at most every
  // kRingReapEveryUs: fewer, larger passes touch the counters the
  // submitting threads update less often.
  const auto t_start = Clock::now();
  const bool short_ =
      c->ring_q_n.load(std::memory_order_relaxed) != 0 ||
      c->ring_pf_n.load(std::memory_order_relaxed) != 0 ||
      c->ring_desc.load(std::memory_order_relaxed) >= c->ring_depth / 2 ||
      c->outstanding.load(std::memory_order_relaxed) >= c->cfg.queue_depth / 2;
  if (!short_ && t_start - c->ring_last_reap <
                     std::chrono::microseconds(kRingReapEveryUs))
    return false;
  c->ring_last_reap = t_start;
  const auto words_before =
      t_start - std::chrono::microseconds(kRingReapWordsAfterUs);
  const uint64_t mask = c->ring_depth - 1;
  const uint64_t published = ms_internal_ring_published(r);
  const bool gone = !ms_internal_ring_alive(r);
  std::vector<RingDone>& batch = c->ring_batch;
  batch.clear();
  uint64_t pos = c->ring_reap_pos, pages = 0;
  while (pos < published) {
    const RingMeta& m = c->ring_meta[pos & mask];
    if (m.seq.load(std::memory_order_acquire) != pos + 1) break;
    const uint64_t end = pos + m.n_pages;
    bool all = m.seen.load(std::memory_order_acquire) == pos + 1;
    if (!all) {
      // left to its client's polls for a while, unless something is short
      if (!short_ && !gone && m.published > words_before) break;
      all = ms_internal_ring_advance(r, end - 1, end) == end;
      for (uint64_t q = pos; q + 1 < end && all; ++q)
        all = ms_internal_ring_advance(r, q, q + 1) == q + 1;
    }
    // once the kernel has ended, what it has not completed never will
    if (!all && !gone) break;
    batch.push_back({m.ticket_slot, m.key_slot, all ? 1 : MS_EDEVICE});
    pages += m.n_pages;
    pos = end;
  }
  if (batch.empty()) return false;
  c->ring_done_pos.store(pos, std::memory_order_release);
  for (const RingDone& d : batch) c->key_refs[d.key_slot].fetch_sub(1);
  {
    std::lock_guard<std::mutex> lk(c->ticket_mu);
    for (const RingDone& d : batch) {
      TicketSlot& t = c->tickets[d.ticket_slot];
      t.state.store(d.state, std::memory_order_release);
      t.ring.store(0, std::memory_order_relaxed);
      c->ticket_free.push_back(d.ticket_slot);
      if (d.state != 1) c->sticky_error.store(MS_EDEVICE);
    }
  }
  const uint64_t n = batch.size();
  c->ring_reap_pos = pos;
  c->outstanding.fetch_sub(n);
  c->st_completed.fetch_add(n);
  c->inflight_bytes.fetch_sub(pages * MS_PAGE_SIZE);
  c->ring_desc.fetch_sub(pages);
  c->ring_reqs.fetch_sub(n);
  c->st_ring_reap_ns.fetch_add(
      (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
          Clock::now() - t_start)
          .count(),
      std::memory_order_relaxed);
  return true;
}

// Move queued small requests onto the ring (caller holds sched_mu): demand
// requests in arrival order while the admission cap and the ring's free
// positions allow, prefetch hints only when no demand request waits and at
// most half the workers hold work, so that a demand request never queues
// behind hints.  True when any request was published or failed.
bool ring_publish(ms_ctx* c) {
  bool any = false;
  if (ensure_ring(c) != MS_OK) {
    // no ring: fail what is queued for it
    std::vector<Pending> gone;
    {
      std::lock_guard<std::mutex> lk(c->q_mu);
      c->ring_q.take(0, true, &gone);
      for (auto& p : c->ring_pf_q) gone.push_back(p);
      c->ring_pf_q.clear();
      c->ring_q_n.store(0, std::memory_order_relaxed);
      c->ring_pf_n.store(0, std::memory_order_relaxed);
    }
    for (auto& p : gone)
      complete_ticket_now(c, p.ticket_slot, MS_EDEVICE,
                          (uint32_t)(p.req.key & 0xffffffffu) - 1);
    return !gone.empty();
  }
  if (c->ring_q_n.load(std::memory_order_relaxed) == 0 &&
      c->ring_pf_n.load(std::memory_order_relaxed) == 0)
    return false;
  ms_resident* r = c->ring.load(std::memory_order_relaxed);
  uint64_t published = 0;
  for (;;) {
    Pending p;
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(c->q_mu);
      if (!c->ring_q.empty()) {
        const Pending& f = c->ring_q.front();
        if (reserve_admission(c, f.req.n_pages * MS_PAGE_SIZE,
                              f.req.n_pages)) {
          p = f;
          c->ring_q.pop_front();
          c->ring_q_n.store(c->ring_q.size(), std::memory_order_relaxed);
          have = true;
        }
      } else if (!c->ring_pf_q.empty() &&
                 c->ring_desc.load() < c->ring_workers / 2) {
        const Pending& f = c->ring_pf_q.front();
        if (reserve_admission(c, f.req.n_pages * MS_PAGE_SIZE,
                              f.req.n_pages)) {
          p = f;
          c->ring_pf_q.pop_front();
          c->ring_pf_n.store(c->ring_pf_q.size(), std::memory_order_relaxed);
          have = true;
        }
      }
    }
    if (!have) break;
    publish_reserved(c, r, p);
    ++published;
    any = true;
  }
  (void)published;
  return any;
}

void scheduler_main(ms_ctx* c) {
  (void)hipSetDevice(c->device);
  auto last_work = Clock::now();
  for (;;) {
    bool did = false, idle_device = true, queues_empty = true;
    // `outstanding` counts requests queued or in flight (a batch's until it
    // is reaped): at zero there is nothing to launch or reap, and the
    // scheduler leaves sched_mu alone, so that a submitting thread finds it
    // free and launches on an idle device itself.  A submission raises the
    // count before it queues, so one the submitter could not launch is seen
    // here on the next pass.
    const bool any = c->outstanding.load(std::memory_order_acquire) != 0;
    if (any) {
      std::lock_guard<std::mutex> lk(c->sched_mu);
      did = reap(c);
      if (c->ring_mode) {
        did = ring_reap(c) || did;
        did = ring_publish(c) || did;
      }
      while (launch_one(c)) did = true;
      idle_device = c->inflight.empty() && c->ring_reqs.load() == 0;
    }
    if (did) {
      last_work = Clock::now();
      continue;
    }
    if (any) {
      std::lock_guard<std::mutex> lk(c->q_mu);
      queues_empty = c->demand_q.empty() && c->prefetch_q.empty() &&
                     c->ring_q.empty() && c->ring_pf_q.empty();
    }
    if (c->stop.load() && queues_empty && idle_device) break;
    if (!idle_device) {
      // work on the device: poll its completion closely
      std::this_thread::yield();
      continue;
    }
    if (!queues_empty) {
      // blocked by admission with nothing in flight cannot happen (a single
      // request never exceeds the cap); just retry
      std::this_thread::yield();
      continue;
    }
    // idle: keep polling for a while (a thread woken from a sleep costs
    // tens of microseconds), then sleep until a submission.  The wake-up
    // test includes `outstanding`: a submission the submitting thread
    // launched itself leaves the queues empty but still has to be reaped.
    if (Clock::now() - last_work <
        std::chrono::microseconds(c->cfg.serve_spin_us)) {
      std::this_thread::yield();
      continue;
    }
    std::unique_lock<std::mutex> lk(c->q_mu);
    c->q_cv.wait_for(lk, std::chrono::milliseconds(2), [c] {
      return c->stop.load() || c->outstanding.load() != 0 ||
             !c->demand_q.empty() || !c->prefetch_q.empty() ||
             !c->ring_q.empty() || !c->ring_pf_q.empty();
    });
  }
}

ms_status alloc_tickets(ms_ctx* c, size_t n, uint32_t* out) {
  std::lock_guard<std::mutex> lk(c->ticket_mu);
  if (c->ticket_free.size() < n) return MS_EAGAIN;
  for (size_t i = 0; i < n; ++i) {
    out[i] = c->ticket_free.back();
    c->ticket_free.pop_back();
    TicketSlot& t = c->tickets[out[i]];
    t.gen.fetch_add(1);
    t.state.store(0);
  }
  return MS_OK;
}

ms_ticket make_ticket(ms_ctx* c, uint32_t slot) {
  return ((uint64_t)c->tickets[slot].gen.load() << 32) | (uint64_t)(slot + 1);
}

ms_status enqueue(ms_ctx* c, const ms_request* reqs, size_t n,
                  ms_ticket* tickets_out, bool prefetch) {
  if (!c) return MS_EINVAL;
  if (c->stop.load()) return MS_ECLOSED;
  if (n == 0) return MS_OK;
  if (!reqs) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  // per-thread scratch, reused from call to call (no allocation per
  // submission once a thread has submitted as many requests at once)
  thread_local std::vector<uint32_t> ks, ts;
  thread_local std::vector<ms_ticket> tk;
  thread_local std::vector<Pending> direct, queued;
  ks.resize(n);
  RangeMemo memo;
  for (size_t i = 0; i < n; ++i) {
    // the handle's liveness is checked below, with the reference taken
    st = check_request(c, reqs[i], &ks[i], false, false, &memo);
    if (st) return st;
    if (reqs[i].n_pages * MS_PAGE_SIZE > c->cfg.admission_cap_bytes)
      return MS_EINVAL;
  }
  const uint64_t prev = c->outstanding.fetch_add(n);
  if (prev + n > c->cfg.queue_depth) {
    c->outstanding.fetch_sub(n);
    if (prefetch) {
      c->st_pf_dropped.fetch_add(n);
      if (tickets_out)
        for (size_t i = 0; i < n; ++i) tickets_out[i] = 0;
      return MS_OK;
    }
    c->st_eagain.fetch_add(1);
    return MS_EAGAIN;
  }
  if (prefetch) {
    std::lock_guard<std::mutex> lk(c->q_mu);
    if (c->prefetch_q.size() + c->ring_pf_q.size() + n >
        c->cfg.prefetch_depth) {
      c->outstanding.fetch_sub(n);
      c->st_pf_dropped.fetch_add(n);
      if (tickets_out)
        for (size_t i = 0; i < n; ++i) tickets_out[i] = 0;
      return MS_OK;
    }
  }
  ts.resize(n);
  st = alloc_tickets(c, n, ts.data());
  if (st) {
    c->outstanding.fetch_sub(n);
    if (prefetch) {
      c->st_pf_dropped.fetch_add(n);
      if (tickets_out)
        for (size_t i = 0; i < n; ++i) tickets_out[i] = 0;
      return MS_OK;
    }
    c->st_eagain.fetch_add(1);
    return st;
  }
  // the tickets are formed now: once a request is published it may finish
  // and its slot be reused (a later generation) before this call returns
  tk.resize(n);
  for (size_t i = 0; i < n; ++i) tk[i] = make_ticket(c, ts[i]);
  // Take a reference on every key under the key lock, re-checking that each
  // handle is still live, so that ms_key_destroy cannot slip in between.
  {
    std::lock_guard<std::mutex> lk(c->key_mu);
    for (size_t i = 0; i < n; ++i) {
      const uint32_t g = (uint32_t)(reqs[i].key >> 32);
      if (!c->key_live[ks[i]] || c->key_gen[ks[i]] != g) {
        st = MS_ENOKEY;
        break;
      }
    }
    if (!st)
      for (size_t i = 0; i < n; ++i) c->key_refs[ks[i]].fetch_add(1);
  }
  if (st) {
    std::lock_guard<std::mutex> lk(c->ticket_mu);
    for (size_t i = 0; i < n; ++i) c->ticket_free.push_back(ts[i]);
    c->outstanding.fetch_sub(n);
    return st;
  }
  // On the ring stage a small request that nothing waits before, and that
  // fits the admission cap and the ring, is published by this thread at
  // once (a reservation is two atomic updates; the ring has its own lock);
  // the others queue for the scheduler.  Whether anything waits is read
  // from the queue sizes without the queue lock; once one of this call's
  // requests queues, the rest queue behind it.
  direct.clear();
  queued.clear();
  ms_resident* ring =
      c->ring_mode ? c->ring.load(std::memory_order_acquire) : nullptr;
  bool ring_queued = false;
  for (size_t i = 0; i < n; ++i) {
    Pending p;
    p.req = reqs[i];
    // store the resolved slot in the low word, generation unchanged
    p.req.key = (reqs[i].key & 0xffffffff00000000ull) | (ks[i] + 1);
    p.ticket_slot = ts[i];
    p.prefetch = prefetch;
    if (c->ring_mode && reqs[i].n_pages <= kRingMaxPages) {
      const bool nothing_waits =
          !ring_queued && c->ring_q_n.load(std::memory_order_relaxed) == 0 &&
          (!prefetch ||
           (c->ring_pf_n.load(std::memory_order_relaxed) == 0 &&
            c->ring_desc.load() < c->ring_workers / 2));
      if (ring && nothing_waits &&
          reserve_admission(c, reqs[i].n_pages * MS_PAGE_SIZE,
                            reqs[i].n_pages)) {
        direct.push_back(p);
        continue;
      }
      ring_queued = true;
    }
    queued.push_back(p);
  }
  uint64_t ring_waiting = 0;
  if (!queued.empty()) {
    std::lock_guard<std::mutex> lk(c->q_mu);
    for (const Pending& p : queued) {
      if (c->ring_mode && p.req.n_pages <= kRingMaxPages && prefetch) {
        c->ring_pf_q.push_back(p);
      } else if (c->ring_mode && p.req.n_pages <= kRingMaxPages) {
        c->ring_q.push(p);
        ++ring_waiting;
      } else
        (prefetch ? c->prefetch_q : c->demand_q).push_back(p);
    }
    c->ring_q_n.store(c->ring_q.size(), std::memory_order_relaxed);
    c->ring_pf_n.store(c->ring_pf_q.size(), std::memory_order_relaxed);
    if (c->ring_q.size() > c->st_ring_max_queued.load(std::memory_order_relaxed))
      c->st_ring_max_queued.store(c->ring_q.size(), std::memory_order_relaxed);
  }
  if (ring_waiting) c->st_ring_queued.fetch_add(ring_waiting);
  if (!direct.empty()) c->st_ring_direct.add(direct.size());
  for (const Pending& p : direct) publish_reserved(c, ring, p);
  if (!prefetch) {
    // direct launch on an idle device: if no batch is in flight and the
    // scheduler is not busy, form and launch the batch on this thread,
    // which saves the hop to the scheduler thread at low load.  Under load
    // (batches in flight) requests queue and the scheduler batches them.
    // Completions are always reaped by the scheduler.
    // On the ring stage the submitting thread publishes its small
    // requests itself whenever the lock is free: a publication is a few
    // stores into mapped memory.
    std::unique_lock<std::mutex> lk(c->sched_mu, std::defer_lock);
    if (direct.size() < n && lk.try_lock() &&
        (c->ring_mode || c->inflight.empty())) {
      int prev = c->device;
      (void)hipGetDevice(&prev);
      if (prev != c->device) (void)hipSetDevice(c->device);
      if (c->ring_mode) (void)ring_publish(c);
      if (c->inflight.empty()) (void)launch_one(c);
      if (prev != c->device) (void)hipSetDevice(prev);
    }
  }
  c->q_cv.notify_one();
  if (!prefetch) c->st_submitted.add(n);
  if (tickets_out)
    for (size_t i = 0; i < n; ++i) tickets_out[i] = tk[i];
  return MS_OK;
}

// One run of pages with one key: the plain kernel with as many waves as stay
// resident (unroll 1), or at most max_waves waves when that is fewer
// (unroll 2).
ms_status launch_plain_run(ms_ctx* c, uint32_t slot, const void* src,
                           void* dst, uint64_t n_pages, const ms_nonce& nonce,
                           hipStream_t s, uint32_t max_waves = 0) {
  ms::PlainArgs a;
  a.keys = c->d_keys;
  a.src = static_cast<const uint8_t*>(src);
  a.dst = static_cast<uint8_t*>(dst);
  a.nonce_array = reinterpret_cast<const uint32_t*>(nonce.array);
  a.nonce_base = nonce.base;
  a.nonce_stride = nonce.stride;
  a.first_page = 0;
  a.n_pages = n_pages;
  a.key_slot = slot;
  a.nonce_tag = nonce.tag;
  const uint32_t kind =
      nonce.kind == MS_NONCE_ARRAY ? ms::kNonceArray : ms::kNonceLinear;
  const Tuning full = plain_tuning(c, false);
  const uint32_t resident = (uint32_t)c->cu_count * full.waves_per_cu;
  const bool capped = max_waves && max_waves < resident;
  const Tuning t = capped ? plain_tuning(c, true) : full;
  return dev_err(c, ms::launch_plain(a, kind, c->cfg.cipher,
                                     (int)c->cfg.rounds,
                                     capped ? max_waves : resident, t.unroll,
                                     s));
}

ms_status plain_call(ms_ctx* c, ms_key key, const void* src, void* dst,
                     uint64_t n_pages, const ms_nonce* nonce, void* stream) {
  if (!c) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  if (n_pages == 0) return MS_OK;
  ms_request r;
  std::memset(&r, 0, sizeof(r));
  r.op = MS_ENCRYPT;
  r.key = key;
  r.src = src;
  r.dst = dst;
  r.n_pages = n_pages;
  if (!nonce) return MS_EINVAL;
  r.nonce = *nonce;
  uint32_t slot = 0;
  st = check_request(c, r, &slot, false);
  if (st) return st;
  if ((st = pin_keys(c, &key, sizeof(ms_key), &slot, 1))) return st;
  KeyPins pins{c, &slot, 1};
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  return launch_plain_run(c, slot, src, dst, n_pages, *nonce, s);
}

ms_status install_key(ms_ctx* c, ms_key* out) {
  // caller holds key_mu and has filled h_staging
  uint32_t slot = UINT32_MAX;
  for (uint32_t i = 0; i < c->cfg.max_keys; ++i)
    if (!c->key_live[i]) {
      slot = i;
      break;
    }
  if (slot == UINT32_MAX) {
    secure_zero(c->h_staging, MS_KEY_BYTES);
    return MS_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(c->d_keys + (size_t)slot * 8, c->h_staging,
                                MS_KEY_BYTES, hipMemcpyHostToDevice, c->stream);
  if (hip_ok(e)) e = hipStreamSynchronize(c->stream);
  secure_zero(c->h_staging, MS_KEY_BYTES);
  if (!hip_ok(e)) return dev_err(c, e);
  c->key_live[slot] = 1;
  uint32_t g = ++c->key_gen[slot];
  if (g == 0) g = ++c->key_gen[slot];
  *out = ((uint64_t)g << 32) | (uint64_t)(slot + 1);
  return MS_OK;
}

}  // namespace

// ================================================================ C ABI ===

extern "C" {

void ms_config_default(ms_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->max_keys = 64;
  cfg->rounds = 20;
  cfg->queue_depth = 65536;
  cfg->max_batch_requests = 1024;
  cfg->admission_cap_bytes = 8ull << 30;
  cfg->inflight_batches = 4;
  cfg->prefetch_depth = 4096;
  cfg->validate_pointers = 1;
  cfg->use_graphs = 1;
  cfg->host_chunk_pages = 16384;
  cfg->host_stage_slots = 3;
  cfg->host_mapped_waves = 128;
  cfg->serve_spin_us = 5000;
}

const char* ms_status_str(ms_status st) {
  switch (st) {
    case MS_OK: return "ok";
    case MS_EINVAL: return "invalid argument";
    case MS_ENOKEY: return "unknown or stale key handle";
    case MS_ENOMEM: return "out of memory or key table full";
    case MS_EAGAIN: return "queue full or admission cap reached";
    case MS_EBUSY: return "key in use by requests in flight";
    case MS_EDEVICE: return "GPU or HIP runtime error";
    case MS_ECLOSED: return "context shutting down";
    case MS_ETIMEDOUT: return "timed out";
    case MS_ENOTSUP: return "not supported";
    case MS_ECANCELED: return "cancelled";
  }
  return "unknown status";
}

ms_status ms_init(ms_ctx** out, int hip_device, const ms_config* cfg_in) {
  if (!out) return MS_EINVAL;
  ms_config cfg;
  if (cfg_in) cfg = *cfg_in; else ms_config_default(&cfg);
  if (cfg.max_keys == 0 || cfg.max_keys > kMaxKeysLimit) return MS_EINVAL;
  if (cfg.rounds != 20 && cfg.rounds != 12 && cfg.rounds != 8)
    return MS_EINVAL;
  if (cfg.cipher != MS_CIPHER_CHACHA && cfg.cipher != MS_CIPHER_SALSA)
    return MS_EINVAL;
  if (cfg.serve_stage > MS_SERVE_STAGE_RING) return MS_EINVAL;
  if (cfg.queue_depth == 0 || (cfg.queue_depth & (cfg.queue_depth - 1)) ||
      cfg.queue_depth > (1u << 24))
    return MS_EINVAL;
  if (cfg.max_batch_requests == 0 || cfg.max_batch_requests > (1u << 20))
    return MS_EINVAL;
  if (cfg.inflight_batches == 0 || cfg.inflight_batches > 64)
    return MS_EINVAL;
  if (cfg.admission_cap_bytes < MS_PAGE_SIZE) return MS_EINVAL;
  if (cfg.host_chunk_pages == 0) cfg.host_chunk_pages = 16384;
  if (cfg.host_stage_slots == 0) cfg.host_stage_slots = 3;
  if (cfg.host_mapped_waves == 0) cfg.host_mapped_waves = 128;
  if (cfg.host_chunk_pages > 65536 || cfg.host_stage_slots < 2 ||
      cfg.host_stage_slots > 16)
    return MS_EINVAL;
  int ndev = 0;
  if (!hip_ok(hipGetDeviceCount(&ndev))) return MS_EDEVICE;
  if (hip_device < 0 || hip_device >= ndev) return MS_EINVAL;
  if (!hip_ok(hipSetDevice(hip_device))) return MS_EDEVICE;

  ms_ctx* c = new (std::nothrow) ms_ctx();
  if (!c) return MS_ENOMEM;
  c->device = hip_device;
  c->cfg = cfg;
  hipDeviceProp_t prop;
  if (!hip_ok(hipGetDeviceProperties(&prop, hip_device))) {
    delete c;
    return MS_EDEVICE;
  }
  c->cu_count = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  c->ring_mode = cfg.serve_stage != MS_SERVE_STAGE_LAUNCH;
  // one workgroup of 4 waves per compute unit: a poller and the workers
  c->ring_workers = (uint32_t)c->cu_count * ms::kWavesPerBlock - 1;
  if (c->ring_mode) {
    c->ring_meta.reset(new (std::nothrow) RingMeta[c->ring_depth]);
    if (!c->ring_meta) {
      delete c;
      return MS_ENOMEM;
    }
  }
  for (uint32_t u = 1; u <= 2; ++u)
    c->resident_plain_wpc[u] = ms::resident_waves_per_cu(
        ms::plain_kernel_fn(u, cfg.cipher, (int)cfg.rounds, ms::kNonceLinear));
  for (uint32_t u = 1; u <= 2; ++u)
    c->resident_batch_wpc[u] =
        ms::resident_waves_per_cu(
            ms::batch_kernel_fn(u, cfg.cipher, (int)cfg.rounds));
  ms_status st = MS_OK;
  const size_t key_bytes = (size_t)cfg.max_keys * MS_KEY_BYTES;
  if (!hip_ok(hipStreamCreate(&c->stream))) st = MS_EDEVICE;
  if (!st && !hip_ok(hipMalloc(reinterpret_cast<void**>(&c->d_keys),
                               key_bytes)))
    st = MS_ENOMEM;
  if (!st && !hip_ok(hipMemset(c->d_keys, 0, key_bytes))) st = MS_EDEVICE;
  if (!st && !hip_ok(hipHostMalloc(reinterpret_cast<void**>(&c->h_staging),
                                   MS_KEY_BYTES, hipHostMallocDefault)))
    st = MS_ENOMEM;
  if (!st && !(c->host = ms_internal_host_path_create())) st = MS_ENOMEM;
  if (!st) {
    secure_zero(c->h_staging, MS_KEY_BYTES);
    c->key_gen.assign(cfg.max_keys, 0);
    c->key_live.assign(cfg.max_keys, 0);
    c->key_refs.reset(new KeyRef[cfg.max_keys]);
    for (uint32_t i = 0; i < cfg.max_keys; ++i) c->key_refs[i].store(0);
    c->tickets = std::vector<TicketSlot>(cfg.queue_depth);
    c->ticket_free.reserve(cfg.queue_depth);
    for (uint32_t i = cfg.queue_depth; i-- > 0;) c->ticket_free.push_back(i);
    c->sync_slots.resize(4);
    for (auto& s : c->sync_slots)
      if (!st) st = alloc_slot(s, cfg.max_batch_requests);
    // ms_process_batch_static: the device array's address on this device
    // (hipGetSymbolAddress, with the device current), its pinned staging
    // and the working storage of its checks
    if (!st && !hip_ok(ms::static_batch_scratch(&c->d_static))) st = MS_EDEVICE;
    if (!st && !hip_ok(hipHostMalloc(reinterpret_cast<void**>(&c->h_static),
                                     ms::kStaticBatchBytes,
                                     hipHostMallocCoherent)))
      st = MS_ENOMEM;
    if (!st && !hip_ok(hipEventCreateWithFlags(&c->static_done,
                                               hipEventDisableTiming)))
      st = MS_EDEVICE;
    if (!st) {
      c->static_slots.resize(MS_STATIC_BATCH_MAX_REQUESTS);
      c->static_ranges.reserve(MS_STATIC_BATCH_MAX_REQUESTS);
    }
    c->serve_slots.resize(cfg.inflight_batches);
    for (auto& s : c->serve_slots)
      if (!st) st = alloc_slot(s, cfg.max_batch_requests);
    c->serve_streams.resize(cfg.inflight_batches, nullptr);
    for (auto& s : c->serve_streams)
      if (!st && !hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)))
        st = MS_EDEVICE;
    for (int i = (int)cfg.inflight_batches; i-- > 0;)
      c->serve_free.push_back(i);
  }
  if (!st) {
    ms_tune_cache_load(c->arch.c_str(), c->cu_count,
                       [c](uint32_t bucket, uint32_t ppw, uint32_t unroll,
                           uint32_t wpc, double us) {
                         Tuning t;
                         t.ppw = ppw;
                         t.unroll = unroll;
                         t.waves_per_cu = wpc;
                         t.us = us;
                         c->tuned[bucket] = t;
                       });
    try {
      c->scheduler = std::thread(scheduler_main, c);
    } catch (...) {
      st = MS_ENOMEM;
    }
  }
  if (st) {
    ms_shutdown(c);
    return st;
  }
  *out = c;
  return MS_OK;
}

ms_status ms_shutdown(ms_ctx* c) {
  if (!c) return MS_OK;
  (void)hipSetDevice(c->device);
  ms_internal_resident_stop_all(c);
  c->stop.store(true);
  c->q_cv.notify_all();
  if (c->scheduler.joinable()) c->scheduler.join();
  // the serving ring's kernel ends once every published request is done
  if (ms_resident* r = c->ring.exchange(nullptr)) ms_internal_ring_stop(r);
  (void)hipDeviceSynchronize();
  if (c->host) ms_internal_host_path_destroy(c->host);
  c->host = nullptr;
  if (c->d_keys) {
    (void)hipMemset(c->d_keys, 0, (size_t)c->cfg.max_keys * MS_KEY_BYTES);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->d_keys);
  }
  if (c->h_staging) {
    secure_zero(c->h_staging, MS_KEY_BYTES);
    (void)hipHostFree(c->h_staging);
  }
  for (auto& s : c->sync_slots) free_slot(s);
  for (auto& s : c->serve_slots) free_slot(s);
  // the device array of ms_process_batch_static stays with the device
  if (c->static_done) (void)hipEventDestroy(c->static_done);
  if (c->h_static) (void)hipHostFree(c->h_static);
  for (auto& s : c->serve_streams)
    if (s) (void)hipStreamDestroy(s);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return MS_OK;
}

ms_status ms_key_load(ms_ctx* c, const uint8_t key[32], ms_key* out) {
  if (!c || !key || !out) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->key_mu);
  std::memcpy(c->h_staging, key, MS_KEY_BYTES);
  return install_key(c, out);
}

ms_status ms_key_generate(ms_ctx* c, ms_key* out) {
  if (!c || !out) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  std::lock_guard<std::mutex> lk(c->key_mu);
  size_t got = 0;
  while (got < MS_KEY_BYTES) {
    ssize_t r = getrandom(c->h_staging + got, MS_KEY_BYTES - got, 0);
    if (r < 0) {
      secure_zero(c->h_staging, MS_KEY_BYTES);
      return MS_EDEVICE;
    }
    got += (size_t)r;
  }
  return install_key(c, out);
}

ms_status ms_key_destroy(ms_ctx* c, ms_key key) {
  if (!c) return MS_EINVAL;
  uint32_t slot = 0;
  if (!resolve_key(c, key, &slot)) return MS_ENOKEY;
  std::lock_guard<std::mutex> lk(c->key_mu);
  if (!c->key_live[slot] || c->key_gen[slot] != (uint32_t)(key >> 32))
    return MS_ENOKEY;
  if (c->key_refs[slot].load() != 0) return MS_EBUSY;
  // stream-ordered launches on any stream may still read the slot
  hipError_t e = hipDeviceSynchronize();
  if (hip_ok(e)) e = hipMemset(c->d_keys + (size_t)slot * 8, 0, MS_KEY_BYTES);
  if (hip_ok(e)) e = hipDeviceSynchronize();
  c->key_live[slot] = 0;
  return dev_err(c, e);
}

ms_status ms_encrypt_pages(ms_ctx* c, ms_key key, const void* src, void* dst,
                           uint64_t n_pages, const ms_nonce* nonce,
                           void* stream) {
  return plain_call(c, key, src, dst, n_pages, nonce, stream);
}

ms_status ms_decrypt_pages(ms_ctx* c, ms_key key, const void* src, void* dst,
                           uint64_t n_pages, const ms_nonce* nonce,
                           void* stream) {
  return plain_call(c, key, src, dst, n_pages, nonce, stream);
}

ms_status ms_plain_launch_info(ms_ctx* c, uint64_t n_pages,
                               int32_t nonce_kind, ms_launch_info* out) {
  if (!c || !out || n_pages == 0) return MS_EINVAL;
  if (nonce_kind != MS_NONCE_ARRAY && nonce_kind != MS_NONCE_LINEAR)
    return MS_EINVAL;
  // the arithmetic of launch_plain_run and ms::launch_plain
  const Tuning t = plain_tuning(c, false);
  const uint64_t max_waves = (uint64_t)c->cu_count * t.waves_per_cu;
  const uint64_t first =
      n_pages < ms::kMaxPagesPerPlainLaunch ? n_pages
                                            : ms::kMaxPagesPerPlainLaunch;
  const uint64_t waves = first < max_waves ? first : max_waves;
  std::memset(out, 0, sizeof(*out));
  const uint32_t kind =
      nonce_kind == MS_NONCE_ARRAY ? ms::kNonceArray : ms::kNonceLinear;
  std::snprintf(out->kernel, sizeof(out->kernel),
                "plain_pages_kernel<%uu, %u, %u, %uu>", c->cfg.cipher,
                c->cfg.rounds, t.unroll, kind);
  out->launches = (uint32_t)((n_pages + ms::kMaxPagesPerPlainLaunch - 1) /
                             ms::kMaxPagesPerPlainLaunch);
  out->grid_blocks =
      (uint32_t)((waves + ms::kWavesPerBlock - 1) / ms::kWavesPerBlock);
  out->block_threads = ms::kBlockThreads;
  out->waves_per_cu = t.waves_per_cu;
  out->cipher = c->cfg.cipher;
  out->rounds = c->cfg.rounds;
  out->unroll = t.unroll;
  out->nonce_kind = (uint32_t)nonce_kind;
  return MS_OK;
}

ms_status ms_process_batch(ms_ctx* c, const ms_request* reqs, size_t n,
                           void* stream) {
  if (!c) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  if (n == 0) return MS_OK;
  if (!reqs || n > c->cfg.max_batch_requests) return MS_EINVAL;
  std::vector<uint32_t> ks(n);
  std::vector<const ms_request*> rp(n);
  RangeMemo memo;
  for (size_t i = 0; i < n; ++i) {
    st = check_request(c, reqs[i], &ks[i], true, true, &memo);
    if (st) return st;
    rp[i] = &reqs[i];
  }
  {
    std::vector<std::pair<uintptr_t, uint64_t>> d;
    d.reserve(n);
    if ((st = check_batch_ranges(reqs, n, d))) return st;
  }
  if ((st = pin_keys(c, &reqs[0].key, sizeof(ms_request), ks.data(), n)))
    return st;
  KeyPins pins{c, ks.data(), n};
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::lock_guard<std::mutex> lk(c->batch_mu);
  BatchSlot& slot = c->sync_slots[c->sync_next];
  c->sync_next = (c->sync_next + 1) % c->sync_slots.size();
  if (slot.used && !hip_ok(hipEventSynchronize(slot.done)))
    return dev_err(c, hipErrorUnknown);
  uint64_t total = 0;
  const size_t copy = fill_slot(slot, rp.data(), ks.data(), n, &total);
  if (!copy) return MS_OK;
  return issue_slot(c, slot, copy, total, s, c->cfg.use_graphs != 0);
}

ms_status ms_process_batch_static(ms_ctx* c, const ms_request* reqs,
                                  size_t n, void* stream) {
  if (!c) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  if (n == 0) return MS_OK;
  if (!reqs || n > MS_STATIC_BATCH_MAX_REQUESTS) return MS_EINVAL;
  if (!c->d_static) return MS_ENOTSUP;
  // everything below uses storage sized at ms_init: no allocation
  std::lock_guard<std::mutex> lk(c->static_mu);
  uint32_t* ks = c->static_slots.data();
  RangeMemo memo;
  for (size_t i = 0; i < n; ++i)
    if ((st = check_request(c, reqs[i], &ks[i], true, true, &memo)))
      return st;
  if ((st = check_batch_ranges(reqs, n, c->static_ranges))) return st;
  if ((st = pin_keys(c, &reqs[0].key, sizeof(ms_request), ks, n))) return st;
  KeyPins pins{c, ks, n};
  // the pinned staging is rewritten only after the previous copy out of it
  // (and the kernel that read the device array) has finished
  if (c->static_used && !hip_ok(hipEventSynchronize(c->static_done)))
    return dev_err(c, hipErrorUnknown);
  uint64_t total = 0;
  const size_t copy = fill_descriptors(
      c->h_static, [reqs](size_t i) -> const ms_request& { return reqs[i]; },
      ks, n, &total);
  if (!copy) return MS_OK;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const Tuning t = tuning_for(c, total);
  const uint32_t grid = grid_blocks_for(c, t, total);
  hipError_t e;
  if (copy <= sizeof(ms::InlineBatch)) {
    // a small batch: one kernel, its records in the kernel arguments
    ms::InlineBatch ib;
    std::memcpy(&ib, c->h_static, copy);
    e = ms::launch_batch_inline(ib, c->d_keys, t.ppw, t.unroll, grid,
                                c->cfg.cipher, (int)c->cfg.rounds, s);
  } else {
    e = ms::launch_desc_copy(c->d_static, c->h_static, copy, s);
    if (hip_ok(e))
      e = ms::launch_batch(static_cast<const ms::DevBatchHdr*>(c->d_static),
                           c->d_keys, t.ppw, t.unroll, grid, c->cfg.cipher,
                           (int)c->cfg.rounds, s);
  }
  if (hip_ok(e)) e = hipEventRecord(c->static_done, s);
  if (!hip_ok(e)) return dev_err(c, e);
  c->static_used = true;
  return MS_OK;
}

ms_status ms_submit(ms_ctx* c, const ms_request* reqs, size_t n,
                    ms_ticket* tickets_out) {
  if (n && !tickets_out) return MS_EINVAL;
  return enqueue(c, reqs, n, tickets_out, false);
}

ms_status ms_prefetch_hint(ms_ctx* c, const ms_request* reqs, size_t n,
                           ms_ticket* tickets_out) {
  return enqueue(c, reqs, n, tickets_out, true);
}

ms_status ms_poll(ms_ctx* c, const ms_ticket* t, size_t n, int32_t* done,
                  uint64_t timeout_ns) {
  if (!c || (n && (!t || !done))) return MS_EINVAL;
  for (size_t i = 0; i < n; ++i) {
    const uint32_t s = (uint32_t)(t[i] & 0xffffffffu);
    if (t[i] != 0 && (s == 0 || s > c->tickets.size())) return MS_EINVAL;
  }
  const auto deadline = Clock::now() + std::chrono::nanoseconds(timeout_ns);
  for (;;) {
    size_t pending = 0;
    for (size_t i = 0; i < n; ++i) {
      if (t[i] == 0) {  // a dropped prefetch hint
        done[i] = MS_ECANCELED;
        continue;
      }
      const uint32_t s = (uint32_t)(t[i] & 0xffffffffu) - 1;
      const uint32_t g = (uint32_t)(t[i] >> 32);
      TicketSlot& ts = c->tickets[s];
      int32_t state = ts.state.load(std::memory_order_acquire);
      if (state == 0) {
        // a request on the ring is done once its positions' completion
        // words say so, before the scheduler reaps it: at once if the
        // reaper's completed prefix covers them, else from the words
        const ms_ticket rt = ts.ring.load(std::memory_order_acquire);
        ms_resident* r = c->ring.load(std::memory_order_acquire);
        if (rt && r) {
          uint64_t first = 0, count = 0;
          ms_internal_ring_span(rt, &first, &count);
          if (first + count <=
              c->ring_done_pos.load(std::memory_order_acquire)) {
            state = 1;
          } else if (ms_internal_ring_done(r, rt)) {
            state = 1;
            // spare the reaper the reads (a stale ticket writes its own
            // position, which no later request at this slot can match)
            c->ring_meta[first & (c->ring_depth - 1)].seen.store(
                first + 1, std::memory_order_release);
          }
        }
      }
      const uint32_t cur = ts.gen.load(std::memory_order_acquire);
      if (cur != g) {
        done[i] = 1;  // slot reused: this ticket completed long ago
      } else {
        done[i] = state;
        if (state == 0) ++pending;
      }
    }
    if (pending == 0) return MS_OK;
    if (Clock::now() >= deadline) return MS_ETIMEDOUT;
    std::this_thread::yield();
  }
}

ms_status ms_cancel_client(ms_ctx* c, uint32_t client, uint64_t* n_out) {
  if (!c) return MS_EINVAL;
  std::vector<Pending> gone;
  {
    std::lock_guard<std::mutex> lk(c->q_mu);
    c->ring_q.take(client, false, &gone);
    for (auto* q : {&c->demand_q, &c->prefetch_q, &c->ring_pf_q}) {
      std::deque<Pending> keep;
      for (auto& p : *q) {
        if (p.req.client == client) gone.push_back(p);
        else keep.push_back(p);
      }
      q->swap(keep);
    }
    c->ring_q_n.store(c->ring_q.size(), std::memory_order_relaxed);
    c->ring_pf_n.store(c->ring_pf_q.size(), std::memory_order_relaxed);
  }
  for (auto& p : gone)
    complete_ticket_now(c, p.ticket_slot, MS_ECANCELED,
                        (uint32_t)(p.req.key & 0xffffffffu) - 1);
  c->st_cancelled.fetch_add(gone.size());
  if (n_out) *n_out = gone.size();
  return MS_OK;
}

ms_status ms_drain(ms_ctx* c, uint64_t timeout_ns) {
  if (!c) return MS_EINVAL;
  const auto deadline = Clock::now() + std::chrono::nanoseconds(timeout_ns);
  while (c->outstanding.load() != 0) {
    if (Clock::now() >= deadline) return MS_ETIMEDOUT;
    std::this_thread::yield();
  }
  return check_sticky(c);
}

ms_status ms_get_tuning(ms_ctx* c, uint64_t n_pages, ms_tuning* out) {
  if (!c || !out) return MS_EINVAL;
  Tuning t = tuning_for(c, n_pages);
  std::memset(out, 0, sizeof(*out));
  out->pages_per_wave = t.ppw;
  out->unroll = t.unroll;
  out->waves_per_cu = t.waves_per_cu;
  out->us_per_launch = t.us;
  return MS_OK;
}

ms_status ms_set_tuning(ms_ctx* c, const ms_tuning* t) {
  if (!c) return MS_EINVAL;
  std::lock_guard<std::mutex> lk(c->tune_mu);
  if (!t) {
    c->forced = false;
    return MS_OK;
  }
  if (t->pages_per_wave == 0 || t->pages_per_wave > 4096 ||
      (t->unroll != 1 && t->unroll != 2) || t->waves_per_cu == 0 ||
      t->waves_per_cu > 256)
    return MS_EINVAL;
  c->forced = true;
  c->forced_tuning.ppw = t->pages_per_wave;
  c->forced_tuning.unroll = t->unroll;
  c->forced_tuning.waves_per_cu = t->waves_per_cu;
  c->forced_tuning.us = 0;
  return MS_OK;
}

ms_status ms_autotune(ms_ctx* c, uint64_t n_pages, ms_tuning* out) {
  if (!c || n_pages == 0 || n_pages > (1ull << 22)) return MS_EINVAL;
  ms_status st = check_sticky(c);
  if (st) return st;
  // scratch batch: 64 requests of mixed sizes summing to n_pages
  const uint64_t bytes = n_pages * MS_PAGE_SIZE;
  uint8_t* buf = nullptr;
  if (!hip_ok(hipMalloc(reinterpret_cast<void**>(&buf), bytes)))
    return MS_ENOMEM;
  BatchSlot slot;
  st = alloc_slot(slot, 64);
  ms_key k = 0;
  if (!st) st = ms_key_generate(c, &k);
  Tuning best;
  best.us = 1e30;
  if (!st) {
    uint32_t slot_idx = (uint32_t)(k & 0xffffffffu) - 1;
    std::vector<ms_request> reqs;
    const uint64_t nreq = std::min<uint64_t>(64, n_pages);
    uint64_t off = 0;
    for (uint64_t i = 0; i < nreq; ++i) {
      // uneven split: request i gets a share growing with i
      uint64_t share = (i + 1 == nreq) ? n_pages - off
                                       : std::max<uint64_t>(1, (n_pages * 2 * (i + 1)) / (nreq * (nreq + 1)));
      if (off + share > n_pages - (nreq - 1 - i)) share = n_pages - (nreq - 1 - i) - off;
      ms_request r;
      std::memset(&r, 0, sizeof(r));
      r.key = k;
      r.src = buf + off * MS_PAGE_SIZE;
      r.dst = buf + off * MS_PAGE_SIZE;
      r.n_pages = share;
      r.nonce.kind = MS_NONCE_LINEAR;
      r.nonce.base = off;
      r.nonce.stride = 1;
      reqs.push_back(r);
      off += share;
    }
    std::vector<const ms_request*> rp;
    std::vector<uint32_t> ks(reqs.size(), slot_idx);
    for (auto& r : reqs) rp.push_back(&r);
    uint64_t total = 0;
    const size_t copy = fill_slot(slot, rp.data(), ks.data(), rp.size(), &total);
    hipError_t he = hipMemcpy(slot.dev, slot.host, copy, hipMemcpyHostToDevice);
    if (!hip_ok(he)) st = dev_err(c, he);
    const uint32_t ppws[] = {1, 2, 4, 8, 16, 32};
    const uint32_t unrolls[] = {1, 2};
    const uint32_t wpcs[] = {8, 16, 24, 32};
    std::vector<Tuning> cands;
    for (uint32_t u : unrolls)
      for (uint32_t ppw : ppws)
        for (uint32_t w : wpcs) {
          if (ppw < u) continue;
          Tuning t;
          t.ppw = ppw;
          t.unroll = u;
          t.waves_per_cu = w;
          cands.push_back(t);
        }
    const auto* hdr = reinterpret_cast<const ms::DevBatchHdr*>(slot.dev);
    auto launch = [&](const Tuning& t) {
      return ms::launch_batch(hdr, c->d_keys, t.ppw, t.unroll,
                              grid_blocks_for(c, t, total), c->cfg.cipher,
                              (int)c->cfg.rounds, c->stream);
    };
    // Under this load the chip settles at a lower clock than it starts
    // with, so a fixed candidate order would favour whichever comes last.
    // The device is first kept busy for about kTuneWarmMs; then every
    // round launches each candidate twice between two events and
    // synchronises once at its end, so that a drift of the clock touches
    // all candidates alike.  A candidate's time is its best round.
    constexpr double kTuneWarmMs = 30.0;
    constexpr int kTuneRounds = 3;
    const auto warm_end =
        Clock::now() + std::chrono::microseconds((int64_t)(kTuneWarmMs * 1e3));
    while (!st && Clock::now() < warm_end) {
      for (int i = 0; i < 8 && hip_ok(he); ++i) he = launch(cands[0]);
      if (hip_ok(he)) he = hipStreamSynchronize(c->stream);
      if (!hip_ok(he)) st = dev_err(c, he);
    }
    std::vector<hipEvent_t> ev(cands.size() + 1, nullptr);
    for (auto& x : ev)
      if (!st && !hip_ok(hipEventCreate(&x))) st = MS_EDEVICE;
    std::vector<float> best_ms(cands.size(), 1e30f);
    for (int round = 0; round < kTuneRounds && !st; ++round) {
      he = hipEventRecord(ev[0], c->stream);
      for (size_t i = 0; i < cands.size() && hip_ok(he); ++i) {
        he = launch(cands[i]);
        if (hip_ok(he)) he = launch(cands[i]);
        if (hip_ok(he)) he = hipEventRecord(ev[i + 1], c->stream);
      }
      if (hip_ok(he)) he = hipEventSynchronize(ev[cands.size()]);
      for (size_t i = 0; i < cands.size() && hip_ok(he); ++i) {
        float ms_ = 0;
        he = hipEventElapsedTime(&ms_, ev[i], ev[i + 1]);
        if (hip_ok(he)) best_ms[i] = std::min(best_ms[i], ms_ / 2);
      }
      if (!hip_ok(he)) st = dev_err(c, he);
    }
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    for (size_t i = 0; i < cands.size() && !st; ++i)
      if (best_ms[i] * 1000.0 < best.us) {
        best = cands[i];
        best.us = best_ms[i] * 1000.0;
      }
  }
  if (k) (void)ms_key_destroy(c, k);
  free_slot(slot);
  (void)hipFree(buf);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lk(c->tune_mu);
    c->tuned[bucket_of(n_pages)] = best;
  }
  ms_tune_cache_store(c->arch.c_str(), c->cu_count, bucket_of(n_pages),
                      best.ppw, best.unroll, best.waves_per_cu, best.us);
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->pages_per_wave = best.ppw;
    out->unroll = best.unroll;
    out->waves_per_cu = best.waves_per_cu;
    out->us_per_launch = best.us;
  }
  return MS_OK;
}

ms_status ms_get_stats(ms_ctx* c, ms_stats* o) {
  if (!c || !o) return MS_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->submitted = c->st_submitted.load();
  o->completed = c->st_completed.load();
  o->rejected_eagain = c->st_eagain.load();
  o->batches = c->st_batches.load();
  o->pages = c->st_pages.load();
  o->prefetch_issued = c->st_pf_issued.load();
  o->prefetch_dropped = c->st_pf_dropped.load();
  o->cancelled = c->st_cancelled.load();
  o->inflight_bytes = c->inflight_bytes.load();
  o->max_inflight_bytes = c->st_max_inflight.load();
  o->max_batch_requests = c->st_max_batch.load();
  o->max_inflight_batches = c->st_max_inflight_batches.load();
  o->ring_direct = c->st_ring_direct.load();
  o->ring_queued = c->st_ring_queued.load();
  o->ring_max_queued = c->st_ring_max_queued.load();
  o->ring_reap_ns = c->st_ring_reap_ns.load();
  return MS_OK;
}

int ms_debug_staging_is_zero(ms_ctx* c) {
  if (!c || !c->h_staging) return -1;
  std::lock_guard<std::mutex> lk(c->key_mu);
  for (uint32_t i = 0; i < MS_KEY_BYTES; ++i)
    if (c->h_staging[i]) return 0;
  return 1;
}

}  // extern "C"

// ------------------------- internal hooks for the other host sources ---

int ms_internal_device(ms_ctx* c) { return c->device; }
int ms_internal_cu_count(ms_ctx* c) { return c->cu_count; }
hipStream_t ms_internal_stream(ms_ctx* c, void* stream) {
  return stream ? static_cast<hipStream_t>(stream) : c->stream;
}
ms_status ms_internal_check_range(ms_ctx* c, const void* p, uint64_t bytes,
                                  uint64_t align) {
  return check_device_range(c, p, bytes, align);
}
ms_status ms_internal_dev_err(ms_ctx* c, hipError_t e) { return dev_err(c, e); }
const ms_config& ms_internal_config(ms_ctx* c) { return c->cfg; }
ms_status ms_internal_sticky(ms_ctx* c) { return check_sticky(c); }
bool ms_internal_resolve_key(ms_ctx* c, ms_key key, uint32_t* slot) {
  return resolve_key(c, key, slot);
}
ms_status ms_internal_pin_key(ms_ctx* c, ms_key key, uint32_t* slot) {
  if (!resolve_key(c, key, slot)) return MS_ENOKEY;
  return pin_keys(c, &key, sizeof(key), slot, 1);
}
void ms_internal_unpin_key(ms_ctx* c, uint32_t slot) {
  unpin_keys(c, &slot, 1);
}
ms_status ms_internal_launch_plain(ms_ctx* c, uint32_t key_slot,
                                   const void* src, void* dst,
                                   uint64_t n_pages, const ms_nonce& nonce,
                                   hipStream_t stream, uint32_t max_waves) {
  return launch_plain_run(c, key_slot, src, dst, n_pages, nonce, stream,
                          max_waves);
}
HostPath* ms_internal_host_path(ms_ctx* c) { return c->host; }
ms_status ms_internal_copy_key(ms_ctx* c, ms_key key, void* dst,
                               hipStream_t stream) {
  // the handle check of resolve_key, made under the lock held for the copy
  // (resolve_key takes the same lock itself)
  const uint32_t s = (uint32_t)(key & 0xffffffffu);
  const uint32_t g = (uint32_t)(key >> 32);
  if (key == 0 || s == 0 || s > c->cfg.max_keys) return MS_ENOKEY;
  std::lock_guard<std::mutex> lk(c->key_mu);
  if (!c->key_live[s - 1] || c->key_gen[s - 1] != g) return MS_ENOKEY;
  const uint32_t slot = s - 1;
  hipError_t e = hipMemcpyAsync(dst, c->d_keys + (size_t)slot * 8,
                                MS_KEY_BYTES, hipMemcpyDeviceToDevice, stream);
  if (hip_ok(e)) e = hipStreamSynchronize(stream);
  return hip_ok(e) ? MS_OK : dev_err(c, e);
}
