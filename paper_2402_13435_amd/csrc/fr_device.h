// Device helpers shared by the HIP sources (fr_kernels.hip, fr_quant.hip).
// Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fr_internal.h"

namespace fr {

// Every launcher refuses a null pointer the kernel would dereference, so a
// host-side wiring mistake becomes an error status instead of a GPU fault.
#define FR_REQUIRE(p) \
  do {                \
    if (!(p)) return hipErrorInvalidValue; \
  } while (0)

static inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 65535u * 4) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------------ order keys
// Scores map to 32-bit keys whose unsigned order is the float order
// (-0 and +0 share a key).  A candidate's 64-bit key appends the complement
// of its id, so the unsigned order of keys is (score desc, id asc) when
// sorted descending.
__device__ __forceinline__ uint32_t fkey(float s) {
  uint32_t u = __float_as_uint(s);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
  if (k <= kKeyNegInf) return -INFINITY;
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

}  // namespace fr
