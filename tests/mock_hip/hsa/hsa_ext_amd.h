// AMD extensions to the mock HSA API (test infrastructure only).
#pragma once
#include "hsa.h"
typedef enum {
  HSA_AMD_AGENT_INFO_BDFID = 0xA006,
  HSA_AMD_AGENT_INFO_DOMAIN = 0xA00F
} hsa_amd_agent_info_t;
