// CPU implementation of the mock HIP runtime of hip/hip_runtime.h (test
// infrastructure only; see that header).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

using Clock = std::chrono::steady_clock;

// ------------------------------------------------------------- streams ---

static std::atomic<uint64_t> g_ops{0};

struct MockStream {
  std::mutex mu;
  std::condition_variable work_cv, idle_cv;
  std::deque<std::function<void()>> q;
  bool stop = false, busy = false;
  std::thread th;

  MockStream() { th = std::thread([this] { run(); }); }
  ~MockStream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    work_cv.notify_all();
    th.join();
  }
  void run() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> lk(mu);
        work_cv.wait(lk, [this] { return stop || !q.empty(); });
        if (q.empty()) return;  // stop requested and drained
        f = std::move(q.front());
        q.pop_front();
        busy = true;
      }
      f();
      g_ops.fetch_add(1);
      {
        std::lock_guard<std::mutex> lk(mu);
        busy = false;
      }
      idle_cv.notify_all();
    }
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back(std::move(f));
    }
    work_cv.notify_one();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    idle_cv.wait(lk, [this] { return q.empty() && !busy; });
  }
};

static std::mutex g_streams_mu;
static std::set<MockStream*> g_streams;

static MockStream* null_stream() {
  static MockStream* s = [] {
    auto* n = new MockStream();
    std::lock_guard<std::mutex> lk(g_streams_mu);
    g_streams.insert(n);
    return n;
  }();
  return s;
}

static MockStream* resolve(hipStream_t s) { return s ? s : null_stream(); }

void mock_enqueue(hipStream_t s, std::function<void()> fn) {
  resolve(s)->push(std::move(fn));
}
uint64_t mock_ops_run() { return g_ops.load(); }

hipError_t hipStreamCreate(hipStream_t* s) {
  if (!s) return hipErrorInvalidValue;
  *s = new MockStream();
  std::lock_guard<std::mutex> lk(g_streams_mu);
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  return hipStreamCreate(s);
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    g_streams.erase(s);
  }
  s->sync();
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  resolve(s)->sync();
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  std::vector<MockStream*> all;
  {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    all.assign(g_streams.begin(), g_streams.end());
  }
  for (MockStream* s : all) s->sync();
  return hipSuccess;
}

// -------------------------------------------------------------- device ---

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d) {
  if (d != 0) return hipErrorInvalidValue;
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->name, "mock");
  std::strcpy(p->gcnArchName, "gfx950-mock");
  // a smaller device for tests that run one host thread per wave
  const char* cus = std::getenv("MOCK_HIP_CUS");
  p->multiProcessorCount = cus ? std::atoi(cus) : 256;
  p->totalGlobalMem = (size_t)1 << 34;
  p->pciBusID = 0x42;  // the mock HSA agent carries the same address
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d) {
  if (d != 0 || a != hipDeviceAttributeWallClockRate) return hipErrorInvalidValue;
  *v = 100000;  // kHz: a 100 MHz wall clock, as the GPU's
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }

// -------------------------------------------------------------- memory ---

struct Alloc {
  size_t size;
  hipMemoryType type;
};
static std::mutex g_mem_mu;
static std::map<uintptr_t, Alloc> g_mem;

static hipError_t track_alloc(void** p, size_t n, hipMemoryType t) {
  if (!p) return hipErrorInvalidValue;
  const size_t sz = n ? n : 1;
  void* q = std::aligned_alloc(256, (sz + 255) & ~(size_t)255);
  if (!q) return hipErrorOutOfMemory;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_mem[reinterpret_cast<uintptr_t>(q)] = Alloc{sz, t};
  *p = q;
  return hipSuccess;
}
static hipError_t track_free(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (!g_mem.erase(reinterpret_cast<uintptr_t>(p))) return hipErrorInvalidValue;
  }
  std::free(p);
  return hipSuccess;
}
static bool find_alloc(const void* p, uintptr_t* base, Alloc* a) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(p);
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_mem.upper_bound(x);
  if (it == g_mem.begin()) return false;
  --it;
  if (x >= it->first + it->second.size) return false;
  *base = it->first;
  *a = it->second;
  return true;
}

hipError_t hipMalloc(void** p, size_t n) {
  return track_alloc(p, n, hipMemoryTypeDevice);
}
hipError_t hipFree(void* p) { return track_free(p); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  return track_alloc(p, n, hipMemoryTypeHost);
}
hipError_t hipHostFree(void* p) { return track_free(p); }

hipError_t hipMemset(void* p, int v, size_t n) {
  null_stream()->sync();
  std::memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t s) {
  resolve(s)->push([p, v, n] { std::memset(p, v, n); });
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  null_stream()->sync();
  std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n,
                          hipMemcpyKind, hipStream_t s) {
  resolve(s)->push([dst, src, n] { std::memmove(dst, src, n); });
  return hipSuccess;
}

hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
  uintptr_t base;
  Alloc al;
  if (!a || !find_alloc(p, &base, &al)) return hipErrorInvalidValue;
  std::memset(a, 0, sizeof(*a));
  a->type = al.type;
  a->device = 0;
  a->devicePointer = const_cast<void*>(p);
  a->hostPointer = al.type == hipMemoryTypeHost ? const_cast<void*>(p) : nullptr;
  return hipSuccess;
}
hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size,
                                 hipDeviceptr_t p) {
  uintptr_t b;
  Alloc al;
  if (!find_alloc(p, &b, &al)) return hipErrorInvalidValue;
  *base = reinterpret_cast<void*>(b);
  *size = al.size;
  return hipSuccess;
}

// -------------------------------------------------------------- events ---

struct MockEvent {
  std::atomic<uint64_t> recorded{0}, done{0};
  std::atomic<int64_t> t_ns{0};
};

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  return hipEventCreate(e);
}
hipError_t hipEventDestroy(hipEvent_t e) {
  // an event may still be pending on a stream: let that finish first
  while (e->done.load() < e->recorded.load()) std::this_thread::yield();
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  const uint64_t seq = e->recorded.fetch_add(1) + 1;
  resolve(s)->push([e, seq] {
    e->t_ns.store(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      Clock::now().time_since_epoch())
                      .count());
    uint64_t cur = e->done.load();
    while (cur < seq && !e->done.compare_exchange_weak(cur, seq)) {
    }
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  return e->done.load() >= e->recorded.load() ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  while (hipEventQuery(e) != hipSuccess) std::this_thread::yield();
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  // the stream's later work waits until the event's recorded work has run
  const uint64_t seq = e->recorded.load();
  resolve(s)->push([e, seq] {
    while (e->done.load() < seq) std::this_thread::yield();
  });
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)((b->t_ns.load() - a->t_ns.load()) / 1e6);
  return hipSuccess;
}

// -------------------------------------------------------------- graphs ---

// Implemented with the mock kernels (mock_kernels.cpp): run one fused
// batch as the kernel node of a graph would.
void mock_run_batch_node(const void* func, const void* hdr,
                         const uint32_t* keys, uint32_t ppw);
namespace ms {
const void* desc_copy_fn();   // mock_kernels.cpp
}

struct MockGraphNode {
  int kind = 0;  // 0 memcpy, 1 kernel
  void* dst = nullptr;
  const void* src = nullptr;
  size_t count = 0;
  const void* func = nullptr;
  const void* hdr = nullptr;
  const uint32_t* keys = nullptr;
  uint32_t ppw = 0;
};
struct MockGraph {
  std::vector<MockGraphNode*> nodes;
};
struct MockGraphExec {
  std::vector<MockGraphNode*> orig;
  std::vector<MockGraphNode> nodes;
};

hipError_t hipGraphCreate(hipGraph_t* g, unsigned) {
  *g = new MockGraph();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  for (auto* n : g->nodes) delete n;
  delete g;
  return hipSuccess;
}
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t* n, hipGraph_t g,
                                   const hipGraphNode_t*, size_t, void* dst,
                                   const void* src, size_t count,
                                   hipMemcpyKind) {
  auto* node = new MockGraphNode();
  node->kind = 0;
  node->dst = dst;
  node->src = src;
  node->count = count;
  g->nodes.push_back(node);
  *n = node;
  return hipSuccess;
}
// The kernels a graph captures: the descriptor copy (dst, src, 16-byte
// units), run as a memmove, and the fused batch kernel (header, key table,
// pages per wave); arguments are taken by value as the runtime does.
bool mock_copy_node_params(const hipKernelNodeParams* p, MockGraphNode* node) {
  if (p->func != ms::desc_copy_fn()) return false;
  node->kind = 0;
  node->dst = *static_cast<void* const*>(p->kernelParams[0]);
  node->src = *static_cast<const void* const*>(p->kernelParams[1]);
  node->count = (size_t)*static_cast<const uint32_t*>(p->kernelParams[2]) * 16;
  return true;
}

hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g,
                                 const hipGraphNode_t*, size_t,
                                 const hipKernelNodeParams* p) {
  auto* node = new MockGraphNode();
  if (mock_copy_node_params(p, node)) {
    g->nodes.push_back(node);
    *n = node;
    return hipSuccess;
  }
  node->kind = 1;
  node->func = p->func;
  node->hdr = *static_cast<const void* const*>(p->kernelParams[0]);
  node->keys = *static_cast<const uint32_t* const*>(p->kernelParams[1]);
  node->ppw = *static_cast<const uint32_t*>(p->kernelParams[2]);
  g->nodes.push_back(node);
  *n = node;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, char*,
                               size_t) {
  auto* x = new MockGraphExec();
  x->orig = g->nodes;
  for (auto* n : g->nodes) x->nodes.push_back(*n);
  *e = x;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t e,
                                             hipGraphNode_t n, void* dst,
                                             const void* src, size_t count,
                                             hipMemcpyKind) {
  for (size_t i = 0; i < e->orig.size(); ++i)
    if (e->orig[i] == n && e->nodes[i].kind == 0) {
      e->nodes[i].dst = dst;
      e->nodes[i].src = src;
      e->nodes[i].count = count;
      return hipSuccess;
    }
  return hipErrorInvalidValue;
}
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t e, hipGraphNode_t n,
                                           const hipKernelNodeParams* p) {
  for (size_t i = 0; i < e->orig.size(); ++i)
    if (e->orig[i] == n) {
      MockGraphNode x;
      if (!mock_copy_node_params(p, &x) || e->nodes[i].kind != 0)
        return hipErrorInvalidValue;   // only the copy node is updated
      e->nodes[i] = x;
      return hipSuccess;
    }
  return hipErrorInvalidValue;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  for (const MockGraphNode& n : e->nodes) {
    if (n.kind == 0) {
      void* dst = n.dst;
      const void* src = n.src;
      const size_t count = n.count;
      resolve(s)->push([dst, src, count] { std::memmove(dst, src, count); });
    } else {
      const MockGraphNode k = n;
      resolve(s)->push(
          [k] { mock_run_batch_node(k.func, k.hdr, k.keys, k.ppw); });
    }
  }
  return hipSuccess;
}
