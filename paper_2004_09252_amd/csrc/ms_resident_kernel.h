// Memory shared between the resident-key kernel (resident.hip) and its host
// side (resident.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

// Most keys one engine holds; its table lives in each workgroup's LDS.
constexpr uint32_t kRkMaxKeys = 64;

// One descriptor of the host's submission ring: a run of pages (at most
// max_pages) in pinned host memory or device memory, ciphered with one of
// the resident keys and the linear rule or an array of nonces.  64 bytes,
// in pinned host memory.
struct RkDesc {
  uint64_t src;           // GPU-visible address of the first source page
  uint64_t dst;           // same for the destination
  uint64_t nonce_base;    // kind 1: nonce of page 0 (state words 13..14);
                          // kind 0: GPU-visible address of page 0's 12
                          // nonce bytes (3 words per page follow)
  uint64_t nonce_stride;  // kind 1: nonce increment per page
  uint64_t seq;           // ring position the descriptor was written for
  uint32_t n_pages;
  uint32_t tag;           // kind 1: state word 15
  uint32_t key;           // index into the engine's keys, < n_keys
  uint32_t kind;          // 0 nonce array, 1 linear nonce (as ms_nonce)
  uint64_t pad;
};
static_assert(sizeof(RkDesc) == 64, "RkDesc layout");

// Control words in pinned host memory.  The host writes `published`,
// `heartbeat` and `stop`; the kernel writes `ready`, `exited` and `error`.
struct RkHostCtl {
  uint64_t published;   // ring positions [0, published) hold descriptors
  uint64_t heartbeat;   // bumped by host calls: counts as activity
  uint32_t stop;        // 1: the kernel ends
  uint32_t ready;       // 1: every worker holds the key, its copy is wiped
  uint32_t exited;      // 1: the poller has left; workers follow
  uint32_t error;       // nonzero: a descriptor failed the kernel's checks
  uint64_t pad[4];
};
static_assert(sizeof(RkHostCtl) == 64, "RkHostCtl layout");

// Control words in device memory, zeroed before the launch.  The published
// count, which the waiting workers poll, has a 128-byte line of its own.
struct RkDevCtl {
  uint64_t published;  // the poller's copy of RkHostCtl::published
  uint64_t pad0[15];
  uint32_t stop;       // poller -> workers
  uint32_t key_loads;  // workers holding the key
  uint64_t pad1[15];
};
static_assert(sizeof(RkDevCtl) == 256, "RkDevCtl layout");

struct RkArgs {
  const RkDesc* ring;     // host, ring_mask + 1 descriptors
  uint64_t* completed;    // host, per slot: position + 1 of the last
                          // descriptor finished in it
  RkHostCtl* hctl;
  RkDevCtl* dctl;
  uint32_t* key_buf;      // device, n_keys x 8 words; wiped once every
                          // worker holds them (registers, or LDS tables)
  uint64_t idle_ticks;    // 100 MHz ticks without host activity before the
                          // kernel ends itself; 0 = no limit
  uint32_t ring_mask;
  uint32_t n_workers;     // worker waves (the poller is one more wave)
  uint32_t max_pages;     // pages per descriptor
  uint32_t n_keys;        // 1: the key stays in every worker's registers;
                          // 2..kRkMaxKeys: a table in each workgroup's LDS;
                          // 0: keys are rows of `key_table` (below)
  uint32_t inv_step;      // worker w serves the positions congruent to
                          // w * inv_step modulo n_workers
  uint32_t table_rows;    // n_keys == 0: rows of key_table
  const uint32_t* key_table;  // n_keys == 0: a context's device key table
                          // (8 words per row), read per descriptor with
                          // system-scope loads; the host keeps a row live
                          // while descriptors that name it are in flight
};

// Kernel entry points (plain C names in the separately built code object),
// one per cipher and round count; launched as (n_workers + 1) waves in 256-thread
// workgroups (the group segment size comes from the code object).
constexpr const char* kResidentKernel20 = "ms_resident_pages_r20.kd";
constexpr const char* kResidentKernel12 = "ms_resident_pages_r12.kd";
constexpr const char* kResidentKernel8 = "ms_resident_pages_r8.kd";
constexpr const char* kResidentSalsa20 = "ms_resident_pages_s20.kd";
constexpr const char* kResidentSalsa12 = "ms_resident_pages_s12.kd";
constexpr const char* kResidentSalsa8 = "ms_resident_pages_s8.kd";

}  // namespace ms
