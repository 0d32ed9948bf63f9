// Pages resident in host memory: include/memshield_host.h, plus the link
// probe of include/memshield_probe.h.
//
// MemShield's server keeps the ciphertext of every protected page in its own
// RAM and hands clear pages to clients in RAM (sections 4.2, 4.3), so each
// cryptographic operation moves its page over the host-GPU link and back.  On
// an MI355X host link the cipher kernel runs about forty times faster than
// the link can feed it; every mode below exists to keep the link busy in both
// directions at once:
//   * mapped: the page kernel's loads and stores go straight to pinned host
//     memory (the kernel is the same one the device-resident calls use);
//   * dma: chunks of pages go host->device on one stream (copy engine), are
//     ciphered in a device staging buffer on a second, and go device->host
//     on a third; chunk k's inbound copy overlaps chunk k-1's kernel and
//     chunk k-2's outbound copy, with a ring of staging buffers guarded by
//     events;
//   * dma_in: the inbound half of dma, the kernel storing to host memory.
#include <hip/hip_runtime.h>
#include <string.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "memshield_host.h"
#include "memshield_probe.h"
#include "ms_internal.h"
#include "ms_kernels.h"

struct HostPath {
  std::mutex alloc_mu;
  std::map<uintptr_t, uint64_t> allocs;  // ms_host_alloc buffers -> bytes

  std::mutex stage_mu;  // staged calls, in enqueue order
  bool staged_ready = false;
  uint64_t chunk_pages = 0;
  hipStream_t s_in = nullptr, s_kernel = nullptr, s_out = nullptr;
  std::vector<uint8_t*> slots;             // device, chunk_pages pages each
  std::vector<hipEvent_t> in_done;         // inbound copy into the slot done
  std::vector<hipEvent_t> kernel_done;     // kernel on the slot done
  std::vector<hipEvent_t> slot_free;       // last use of the slot done
  hipEvent_t entry = nullptr;              // caller's stream at entry
  hipEvent_t exit_kernel = nullptr, exit_out = nullptr;
};

namespace {

enum class Where { kDevice, kHost };

struct Buf {
  Where where;
  const uint8_t* host;  // the caller's address
  const uint8_t* gpu;   // the address the GPU uses for it
};

bool hip_ok(hipError_t e) { return e == hipSuccess; }

// Classify [p, p+bytes): device memory of the context's device, or pinned
// host memory mapped into the GPU's address space.  With pointer validation
// on, the range must lie inside the allocation that holds p.
ms_status classify(ms_ctx* c, const void* p, uint64_t bytes, uint64_t align,
                   Buf* out) {
  if (!p || reinterpret_cast<uintptr_t>(p) % align) return MS_EINVAL;
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  if (!hip_ok(hipPointerGetAttributes(&attr, p))) {
    (void)hipGetLastError();
    return MS_EINVAL;
  }
  const uint8_t* q = static_cast<const uint8_t*>(p);
  if (attr.type == hipMemoryTypeDevice) {
    ms_status st = ms_internal_check_range(c, p, bytes, align);
    if (st) return st;
    *out = {Where::kDevice, q, q};
    return MS_OK;
  }
  if (attr.type != hipMemoryTypeHost || !attr.devicePointer ||
      !attr.hostPointer)
    return MS_EINVAL;  // pageable, managed or unknown memory
  if (ms_internal_config(c).validate_pointers) {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (!hip_ok(hipMemGetAddressRange(&base, &size, const_cast<void*>(p)))) {
      (void)hipGetLastError();
      return MS_EINVAL;
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if (a < b || bytes > size || a - b > size - bytes) return MS_EINVAL;
  }
  const uint8_t* hb = static_cast<const uint8_t*>(attr.hostPointer);
  const uint8_t* db = static_cast<const uint8_t*>(attr.devicePointer);
  *out = {Where::kHost, q, db + (q - hb)};
  return MS_OK;
}

// The nonce of page `first` of a run, as the nonce of page 0 of a sub-run.
ms_nonce nonce_at(const ms_nonce& n, uint64_t first) {
  ms_nonce r = n;
  if (n.kind == MS_NONCE_ARRAY)
    r.array = n.array + first * MS_NONCE_BYTES;
  else
    r.base = n.base + first * n.stride;  // modulo 2^64, as for page `first`
  return r;
}

void release_staged(HostPath* h) {
  for (auto* v : {&h->in_done, &h->kernel_done, &h->slot_free})
    for (hipEvent_t e : *v)
      if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {h->entry, h->exit_kernel, h->exit_out})
    if (e) (void)hipEventDestroy(e);
  for (uint8_t* s : h->slots)
    if (s) {
      (void)hipMemset(s, 0, h->chunk_pages * MS_PAGE_SIZE);
      (void)hipDeviceSynchronize();
      (void)hipFree(s);
    }
  for (hipStream_t s : {h->s_in, h->s_kernel, h->s_out})
    if (s) (void)hipStreamDestroy(s);
  h->in_done.clear();
  h->kernel_done.clear();
  h->slot_free.clear();
  h->slots.clear();
  h->entry = h->exit_kernel = h->exit_out = nullptr;
  h->s_in = h->s_kernel = h->s_out = nullptr;
  h->staged_ready = false;
}

// Streams, events and staging buffers of the staged modes, on first use.
// Caller holds stage_mu.
ms_status ensure_staged(ms_ctx* c, HostPath* h) {
  if (h->staged_ready) return MS_OK;
  const ms_config& cfg = ms_internal_config(c);
  h->chunk_pages = cfg.host_chunk_pages;
  const uint32_t n = cfg.host_stage_slots;
  bool ok = true;
  for (hipStream_t* s : {&h->s_in, &h->s_kernel, &h->s_out})
    ok = ok && hip_ok(hipStreamCreateWithFlags(s, hipStreamNonBlocking));
  for (hipEvent_t* e : {&h->entry, &h->exit_kernel, &h->exit_out})
    ok = ok && hip_ok(hipEventCreateWithFlags(e, hipEventDisableTiming));
  h->slots.assign(n, nullptr);
  h->in_done.assign(n, nullptr);
  h->kernel_done.assign(n, nullptr);
  h->slot_free.assign(n, nullptr);
  bool mem_ok = true;
  for (uint32_t i = 0; ok && mem_ok && i < n; ++i) {
    mem_ok = hip_ok(hipMalloc(reinterpret_cast<void**>(&h->slots[i]),
                              h->chunk_pages * MS_PAGE_SIZE));
    if (!mem_ok) {
      h->slots[i] = nullptr;
      (void)hipGetLastError();
      break;
    }
    for (auto* v : {&h->in_done, &h->kernel_done, &h->slot_free})
      ok = ok && hip_ok(hipEventCreateWithFlags(&(*v)[i],
                                                hipEventDisableTiming));
  }
  if (ok && mem_ok) {
    h->staged_ready = true;
    return MS_OK;
  }
  release_staged(h);
  return mem_ok ? MS_EDEVICE : MS_ENOMEM;
}

// The chunk pipeline.  Slot i's buffer is written first by the inbound copy
// (stage_in) or by the kernel (stage_out only) and last used by the outbound
// copy (stage_out) or the kernel; its first writer waits for slot_free[i],
// recorded after its last use, so a slot is reused only when drained, also
// across calls.
ms_status run_staged(ms_ctx* c, HostPath* h, uint32_t key_slot,
                     const Buf& src, const Buf& dst, uint64_t n_pages,
                     const ms_nonce& nonce, bool stage_in, bool stage_out,
                     hipStream_t caller) {
  std::lock_guard<std::mutex> lk(h->stage_mu);
  ms_status st = ensure_staged(c, h);
  if (st) return st;
  hipError_t e = hipEventRecord(h->entry, caller);
  for (hipStream_t s : {h->s_in, h->s_kernel, h->s_out})
    if (hip_ok(e)) e = hipStreamWaitEvent(s, h->entry, 0);
  const uint64_t chunk = h->chunk_pages;
  const size_t n_slots = h->slots.size();
  uint64_t k = 0;
  for (uint64_t first = 0; hip_ok(e) && first < n_pages; first += chunk, ++k) {
    const uint64_t pages = n_pages - first < chunk ? n_pages - first : chunk;
    const size_t bytes = pages * MS_PAGE_SIZE;
    const size_t off = first * MS_PAGE_SIZE;
    const size_t i = k % n_slots;
    uint8_t* buf = h->slots[i];
    if (stage_in) {
      e = hipStreamWaitEvent(h->s_in, h->slot_free[i], 0);
      if (hip_ok(e))
        e = hipMemcpyAsync(buf, src.host + off, bytes, hipMemcpyHostToDevice,
                           h->s_in);
      if (hip_ok(e)) e = hipEventRecord(h->in_done[i], h->s_in);
      if (hip_ok(e)) e = hipStreamWaitEvent(h->s_kernel, h->in_done[i], 0);
    } else {
      e = hipStreamWaitEvent(h->s_kernel, h->slot_free[i], 0);
    }
    if (!hip_ok(e)) break;
    const void* kin = stage_in ? static_cast<const void*>(buf)
                               : static_cast<const void*>(src.gpu + off);
    void* kout = stage_out ? static_cast<void*>(buf)
                           : const_cast<uint8_t*>(dst.gpu + off);
    // a kernel that stores to host memory is bound by the link
    const uint32_t waves =
        stage_out || dst.where != Where::kHost
            ? 0
            : ms_internal_config(c).host_mapped_waves;
    st = ms_internal_launch_plain(c, key_slot, kin, kout, pages,
                                  nonce_at(nonce, first), h->s_kernel, waves);
    if (st) return st;
    if (stage_out) {
      e = hipEventRecord(h->kernel_done[i], h->s_kernel);
      if (hip_ok(e)) e = hipStreamWaitEvent(h->s_out, h->kernel_done[i], 0);
      if (hip_ok(e))
        e = hipMemcpyAsync(const_cast<uint8_t*>(dst.host) + off, buf, bytes,
                           hipMemcpyDeviceToHost, h->s_out);
      if (hip_ok(e)) e = hipEventRecord(h->slot_free[i], h->s_out);
    } else {
      e = hipEventRecord(h->slot_free[i], h->s_kernel);
    }
  }
  // the caller's stream continues after the last kernel and the last copy
  if (hip_ok(e)) e = hipEventRecord(h->exit_kernel, h->s_kernel);
  if (hip_ok(e)) e = hipStreamWaitEvent(caller, h->exit_kernel, 0);
  if (hip_ok(e) && stage_out) e = hipEventRecord(h->exit_out, h->s_out);
  if (hip_ok(e) && stage_out) e = hipStreamWaitEvent(caller, h->exit_out, 0);
  return ms_internal_dev_err(c, e);
}

ms_status host_call(ms_ctx* c, ms_key key, const void* src, void* dst,
                    uint64_t n_pages, const ms_nonce* nonce, int32_t mode,
                    void* stream) {
  if (!c) return MS_EINVAL;
  ms_status st = ms_internal_sticky(c);
  if (st) return st;
  if (mode < MS_HOST_AUTO || mode > MS_HOST_DMA_IN) return MS_EINVAL;
  if (n_pages == 0) return MS_OK;
  if (!nonce || n_pages > UINT64_MAX / MS_PAGE_SIZE) return MS_EINVAL;
  const uint64_t bytes = n_pages * MS_PAGE_SIZE;
  Buf s{}, d{};
  if ((st = classify(c, src, bytes, 16, &s))) return st;
  // in place: the same range, already classified
  if (dst == src)
    d = s;
  else if ((st = classify(c, dst, bytes, 16, &d)))
    return st;
  const uintptr_t a = reinterpret_cast<uintptr_t>(src);
  const uintptr_t b = reinterpret_cast<uintptr_t>(dst);
  if (a != b && a < b + bytes && b < a + bytes) return MS_EINVAL;
  if (nonce->kind == MS_NONCE_ARRAY) {
    if (n_pages > UINT64_MAX / MS_NONCE_BYTES) return MS_EINVAL;
    if ((st = ms_internal_check_range(c, nonce->array,
                                      n_pages * MS_NONCE_BYTES, 4)))
      return st;
  } else if (nonce->kind != MS_NONCE_LINEAR) {
    return MS_EINVAL;
  }
  uint32_t slot = 0;
  if ((st = ms_internal_pin_key(c, key, &slot))) return st;
  // released once the launches below are enqueued (or failed)
  struct Unpin {
    ms_ctx* c;
    uint32_t slot;
    ~Unpin() { ms_internal_unpin_key(c, slot); }
  } unpin{c, slot};
  // Measured on an MI355X host link (host -> host, 1 MiB to 4 GiB): the
  // mapped kernel with host_mapped_waves = 128 matches or passes the staged
  // pipeline at every size (49 GB/s against 47-48 from 1 GiB up, 40 against
  // 25 at 16 MiB) and has the lowest latency.
  if (mode == MS_HOST_AUTO) mode = MS_HOST_MAPPED;
  const bool stage_in =
      s.where == Where::kHost && (mode == MS_HOST_DMA || mode == MS_HOST_DMA_IN);
  const bool stage_out = d.where == Where::kHost && mode == MS_HOST_DMA;
  hipStream_t caller = ms_internal_stream(c, stream);
  if (!stage_in && !stage_out) {
    // a kernel that reads or writes host memory is bound by the link, not
    // by residency: fewer waves keep fewer reads outstanding on it
    const bool on_link = s.where == Where::kHost || d.where == Where::kHost;
    const uint32_t waves = on_link ? ms_internal_config(c).host_mapped_waves
                                   : 0;
    return ms_internal_launch_plain(c, slot, s.gpu, const_cast<uint8_t*>(d.gpu),
                                    n_pages, *nonce, caller, waves);
  }
  return run_staged(c, ms_internal_host_path(c), slot, s, d, n_pages, *nonce,
                    stage_in, stage_out, caller);
}

}  // namespace

ms_status ms_internal_classify_host(ms_ctx* c, const void* p, uint64_t bytes,
                                    uint64_t align, uint64_t* gpu) {
  Buf b{};
  ms_status st = classify(c, p, bytes, align, &b);
  if (st) return st;
  if (b.where != Where::kHost) return MS_EINVAL;
  *gpu = reinterpret_cast<uint64_t>(b.gpu);
  return MS_OK;
}

ms_status ms_internal_classify_any(ms_ctx* c, const void* p, uint64_t bytes,
                                   uint64_t align, uint64_t* gpu) {
  Buf b{};
  ms_status st = classify(c, p, bytes, align, &b);
  if (st) return st;
  *gpu = reinterpret_cast<uint64_t>(b.gpu);
  return MS_OK;
}

HostPath* ms_internal_host_path_create() {
  return new (std::nothrow) HostPath();
}

void ms_internal_host_path_destroy(HostPath* h) {
  if (!h) return;
  release_staged(h);
  for (auto& kv : h->allocs) {
    explicit_bzero(reinterpret_cast<void*>(kv.first), kv.second);
    (void)hipHostFree(reinterpret_cast<void*>(kv.first));
  }
  delete h;
}

extern "C" {

ms_status ms_host_alloc(ms_ctx* c, uint64_t bytes, void** out) {
  if (!c || !out || bytes == 0) return MS_EINVAL;
  HostPath* h = ms_internal_host_path(c);
  void* p = nullptr;
  // coherent (fine-grained): a running kernel may read what the host writes
  // and the other way round, without a dispatch boundary in between
  if (!hip_ok(hipHostMalloc(&p, bytes, hipHostMallocCoherent)) || !p) {
    (void)hipGetLastError();
    return MS_ENOMEM;
  }
  std::memset(p, 0, bytes);
  try {
    std::lock_guard<std::mutex> lk(h->alloc_mu);
    h->allocs[reinterpret_cast<uintptr_t>(p)] = bytes;
  } catch (...) {
    (void)hipHostFree(p);
    return MS_ENOMEM;
  }
  *out = p;
  return MS_OK;
}

ms_status ms_host_free(ms_ctx* c, void* p) {
  if (!c || !p) return MS_EINVAL;
  HostPath* h = ms_internal_host_path(c);
  uint64_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(h->alloc_mu);
    auto it = h->allocs.find(reinterpret_cast<uintptr_t>(p));
    if (it == h->allocs.end()) return MS_EINVAL;
    bytes = it->second;
    h->allocs.erase(it);
  }
  explicit_bzero(p, bytes);
  return hip_ok(hipHostFree(p)) ? MS_OK : MS_EDEVICE;
}

ms_status ms_encrypt_host_pages(ms_ctx* c, ms_key key, const void* src,
                                void* dst, uint64_t n_pages,
                                const ms_nonce* nonce, int32_t mode,
                                void* stream) {
  return host_call(c, key, src, dst, n_pages, nonce, mode, stream);
}

ms_status ms_decrypt_host_pages(ms_ctx* c, ms_key key, const void* src,
                                void* dst, uint64_t n_pages,
                                const ms_nonce* nonce, int32_t mode,
                                void* stream) {
  return host_call(c, key, src, dst, n_pages, nonce, mode, stream);
}

ms_status ms_probe_link(ms_ctx* c, const void* src, void* dst, uint64_t bytes,
                        int32_t engine, void* stream) {
  if (!c || bytes == 0 || bytes % 16 || (engine != 0 && engine != 1))
    return MS_EINVAL;
  Buf s{}, d{};
  ms_status st = classify(c, src, bytes, 16, &s);
  if (st) return st;
  if ((st = classify(c, dst, bytes, 16, &d))) return st;
  const uintptr_t a = reinterpret_cast<uintptr_t>(src);
  const uintptr_t b = reinterpret_cast<uintptr_t>(dst);
  if (a < b + bytes && b < a + bytes) return MS_EINVAL;
  hipStream_t hs = ms_internal_stream(c, stream);
  if (engine == 0)
    return ms_internal_dev_err(
        c, ms::launch_copy(s.gpu, const_cast<uint8_t*>(d.gpu), bytes, 0, hs));
  return ms_internal_dev_err(
      c, hipMemcpyAsync(const_cast<uint8_t*>(d.host), s.host, bytes,
                        hipMemcpyDefault, hs));
}

}  // extern "C"
