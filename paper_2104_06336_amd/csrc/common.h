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
// sum over the 64 lanes of a wave with DPP lane moves (all lanes must be active); the total is
// returned to every lane (read from lane 63).  quad_perm [1,0,3,2] and [2,3,0,1] give quad sums,
// row_half_mirror and row_mirror row (16-lane) sums, row_bcast15 / row_bcast31 carry rows 0 and
// 2 into 1 and 3, then rows 0-1 into 2-3.
__device__ __forceinline__ int wave_sum_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return __builtin_amdgcn_readlane(v, 63);
}

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

// Workgroups of the kernel `fn` (launched with `threads` threads and `lds` bytes of dynamic LDS)
// that the current device holds at once, remembered per (kernel, device, LDS size); 0 if the
// runtime cannot tell.  A grid-stride kernel launched with this many workgroups keeps every
// workgroup resident for the whole launch.
int resident_blocks(const void* fn, int threads, size_t lds = 0);

}  // namespace stem
