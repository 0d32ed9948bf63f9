// Persistent cache of autotuned batch tilings (internal).
#pragma once

#include <stdint.h>

#include <functional>

// Calls `fn(bucket, pages_per_wave, unroll, waves_per_cu, us)` for every
// entry of the cache file named by $MS_TUNE_CACHE that matches the device.
void ms_tune_cache_load(
    const char* arch, int cu_count,
    const std::function<void(uint32_t, uint32_t, uint32_t, uint32_t, double)>&
        fn);

// Adds or replaces one entry in $MS_TUNE_CACHE (no-op when unset).
void ms_tune_cache_store(const char* arch, int cu_count, uint32_t bucket,
                         uint32_t ppw, uint32_t unroll, uint32_t waves_per_cu,
                         double us);
