// A CPU stand-in for the part of the HSA runtime API that the resident-key
// engine's host code (resident.cpp) uses (test infrastructure only; see
// hip/hip_runtime.h beside it).  A kernel-dispatch packet rung on a mock
// queue's doorbell starts mock_hsa.cpp's CPU model of the resident-key
// kernel instead of GPU code.
#pragma once

#include <stddef.h>
#include <stdint.h>

typedef enum {
  HSA_STATUS_SUCCESS = 0,
  HSA_STATUS_INFO_BREAK = 1,
  HSA_STATUS_ERROR = 0x1000
} hsa_status_t;

typedef struct hsa_agent_s { uint64_t handle; } hsa_agent_t;
typedef struct hsa_signal_s { uint64_t handle; } hsa_signal_t;
typedef struct hsa_code_object_reader_s { uint64_t handle; } hsa_code_object_reader_t;
typedef struct hsa_executable_s { uint64_t handle; } hsa_executable_t;
typedef struct hsa_executable_symbol_s { uint64_t handle; } hsa_executable_symbol_t;
typedef int64_t hsa_signal_value_t;

typedef enum { HSA_DEVICE_TYPE_CPU = 0, HSA_DEVICE_TYPE_GPU = 1 } hsa_device_type_t;
typedef enum {
  HSA_AGENT_INFO_DEVICE = 17,
  HSA_AGENT_INFO_QUEUE_MIN_SIZE = 13
} hsa_agent_info_t;
typedef enum { HSA_PROFILE_FULL = 1 } hsa_profile_t;
typedef enum { HSA_DEFAULT_FLOAT_ROUNDING_MODE_DEFAULT = 0 } hsa_default_float_rounding_mode_t;
typedef enum {
  HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT = 22,
  HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE = 11,
  HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE = 13,
  HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE = 14
} hsa_executable_symbol_info_t;
typedef enum { HSA_QUEUE_TYPE_MULTI = 0, HSA_QUEUE_TYPE_SINGLE = 1 } hsa_queue_type32_t;
typedef enum { HSA_SIGNAL_CONDITION_EQ = 0, HSA_SIGNAL_CONDITION_NE = 1,
               HSA_SIGNAL_CONDITION_LT = 2, HSA_SIGNAL_CONDITION_GTE = 3 } hsa_signal_condition_t;
typedef enum { HSA_WAIT_STATE_BLOCKED = 0, HSA_WAIT_STATE_ACTIVE = 1 } hsa_wait_state_t;
enum { HSA_PACKET_TYPE_KERNEL_DISPATCH = 2 };
enum { HSA_PACKET_HEADER_TYPE = 0, HSA_PACKET_HEADER_BARRIER = 8,
       HSA_PACKET_HEADER_SCACQUIRE_FENCE_SCOPE = 9,
       HSA_PACKET_HEADER_SCRELEASE_FENCE_SCOPE = 11 };
enum { HSA_FENCE_SCOPE_SYSTEM = 2 };
enum { HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS = 0 };

typedef struct hsa_queue_s {
  uint32_t type;
  uint32_t features;
  void* base_address;
  hsa_signal_t doorbell_signal;
  uint32_t size;
  uint32_t reserved1;
  uint64_t id;
} hsa_queue_t;

typedef struct hsa_kernel_dispatch_packet_s {
  uint16_t header;
  uint16_t setup;
  uint16_t workgroup_size_x, workgroup_size_y, workgroup_size_z;
  uint16_t reserved0;
  uint32_t grid_size_x, grid_size_y, grid_size_z;
  uint32_t private_segment_size;
  uint32_t group_segment_size;
  uint64_t kernel_object;
  void* kernarg_address;
  uint64_t reserved2;
  hsa_signal_t completion_signal;
} hsa_kernel_dispatch_packet_t;

hsa_status_t hsa_init();
hsa_status_t hsa_shut_down();
hsa_status_t hsa_iterate_agents(hsa_status_t (*cb)(hsa_agent_t, void*), void* data);
hsa_status_t hsa_agent_get_info(hsa_agent_t a, hsa_agent_info_t attr, void* value);
hsa_status_t hsa_code_object_reader_create_from_memory(const void* code, size_t size,
                                                       hsa_code_object_reader_t* r);
hsa_status_t hsa_code_object_reader_destroy(hsa_code_object_reader_t r);
hsa_status_t hsa_executable_create_alt(hsa_profile_t p, hsa_default_float_rounding_mode_t m,
                                       const char* options, hsa_executable_t* e);
hsa_status_t hsa_executable_load_agent_code_object(hsa_executable_t e, hsa_agent_t a,
                                                   hsa_code_object_reader_t r,
                                                   const char* options, void* loaded);
hsa_status_t hsa_executable_freeze(hsa_executable_t e, const char* options);
hsa_status_t hsa_executable_get_symbol_by_name(hsa_executable_t e, const char* name,
                                               const hsa_agent_t* a,
                                               hsa_executable_symbol_t* s);
hsa_status_t hsa_executable_symbol_get_info(hsa_executable_symbol_t s,
                                            hsa_executable_symbol_info_t attr, void* value);
hsa_status_t hsa_executable_destroy(hsa_executable_t e);
hsa_status_t hsa_queue_create(hsa_agent_t a, uint32_t size, hsa_queue_type32_t type,
                              void (*cb)(hsa_status_t, hsa_queue_t*, void*), void* data,
                              uint32_t private_size, uint32_t group_size, hsa_queue_t** q);
hsa_status_t hsa_queue_destroy(hsa_queue_t* q);
uint64_t hsa_queue_add_write_index_relaxed(const hsa_queue_t* q, uint64_t value);
hsa_status_t hsa_signal_create(hsa_signal_value_t initial, uint32_t num_consumers,
                               const hsa_agent_t* consumers, hsa_signal_t* s);
hsa_status_t hsa_signal_destroy(hsa_signal_t s);
void hsa_signal_store_screlease(hsa_signal_t s, hsa_signal_value_t v);
hsa_signal_value_t hsa_signal_wait_scacquire(hsa_signal_t s, hsa_signal_condition_t c,
                                             hsa_signal_value_t compare, uint64_t timeout_hint,
                                             hsa_wait_state_t state);
