// Calibration probes behind include/memshield_probe.h.
#include <hip/hip_runtime.h>

#include "memshield_probe.h"
#include "ms_internal.h"
#include "ms_kernels.h"

extern "C" {

ms_status ms_probe_copy(ms_ctx* c, const void* src, void* dst, uint64_t bytes,
                        uint32_t grid_blocks, void* stream) {
  if (!c || bytes == 0 || bytes % 16) return MS_EINVAL;
  ms_status st = ms_internal_check_range(c, src, bytes, 16);
  if (st) return st;
  st = ms_internal_check_range(c, dst, bytes, 16);
  if (st) return st;
  const uintptr_t s = reinterpret_cast<uintptr_t>(src);
  const uintptr_t d = reinterpret_cast<uintptr_t>(dst);
  if (s < d + bytes && d < s + bytes) return MS_EINVAL;
  if (grid_blocks == 0) grid_blocks = 8u * (uint32_t)ms_internal_cu_count(c);
  return ms_internal_dev_err(
      c, ms::launch_copy(src, dst, bytes, grid_blocks,
                         ms_internal_stream(c, stream)));
}

ms_status ms_probe_valu(ms_ctx* c, uint32_t* out, uint32_t iters,
                        uint32_t grid_blocks, void* stream, uint64_t* ops_out) {
  if (!c || iters == 0) return MS_EINVAL;
  if (grid_blocks == 0) grid_blocks = 32u * (uint32_t)ms_internal_cu_count(c);
  ms_status st = ms_internal_check_range(
      c, out, (uint64_t)grid_blocks * ms::kBlockThreads * 4u, 4);
  if (st) return st;
  st = ms_internal_dev_err(c, ms::launch_valu(out, iters, grid_blocks,
                                              ms_internal_stream(c, stream)));
  if (st) return st;
  if (ops_out) *ops_out = ms::valu_probe_ops(iters, grid_blocks);
  return MS_OK;
}

int ms_device_cu_count(ms_ctx* c) { return c ? ms_internal_cu_count(c) : -1; }

}  // extern "C"
