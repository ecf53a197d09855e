// Shared internals of the stem4d HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stem4d.h"

namespace stem {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------------
// complex helpers (float2 = re, im)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }
// multiply by +i
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }

// ---------------------------------------------------------------------------------------------
// status reporting: device-side error bits are OR-ed into the caller's status word

__device__ __forceinline__ void report(int32_t* status, int32_t bits) {
  if (status != nullptr && bits != 0) atomicOr(status, bits);
}

// ---------------------------------------------------------------------------------------------
// host helpers

inline bool is_pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

#define STEM_HIP_CHECK(expr)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return STEM_EHIP;      \
  } while (0)

#define STEM_LAUNCH_CHECK()                      \
  do {                                           \
    hipError_t e_ = hipGetLastError();           \
    if (e_ != hipSuccess) return STEM_EHIP;      \
  } while (0)

}  // namespace stem
