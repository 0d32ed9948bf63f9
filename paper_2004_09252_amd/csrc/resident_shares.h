// How the resident-key kernel's workers share the ring positions (host
// side; resident.hip applies the result).  Plain C++, no device code.
#pragma once

#include <stdint.h>

namespace ms {

// Worker w of `workers` owns the ring positions congruent to w * inverse
// modulo `workers`, so position q belongs to worker (q mod workers) * step
// mod workers, where step is the smallest integer >= 4 coprime to
// `workers`: consecutive positions then fall in different workgroups of 4
// waves.  Returns that inverse (0 for a single worker).
inline uint32_t share_stride_inverse(uint32_t workers) {
  if (workers <= 1) return 0;
  auto gcd = [](uint64_t x, uint64_t y) {
    while (y) {
      const uint64_t t = x % y;
      x = y;
      y = t;
    }
    return x;
  };
  uint64_t step = 4;
  while (gcd(step, workers) != 1) ++step;
  step %= workers;
  for (uint64_t inv = 1; inv < workers; ++inv)
    if (step * inv % workers == 1) return (uint32_t)inv;
  return 1;  // not reached: step is a unit modulo workers
}

}  // namespace ms
