// Detector / scan geometry shared by host and device code: exact integer division by an
// invariant divisor, the kept-bin predicate and the per-row description of the kept set.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stem4d.h"

namespace stem {

// floor(n / d) for 0 <= n < 2^31 and 1 <= d < 2^31 by one 64-bit multiply and shift:
// with l = ceil(log2 d), m = ceil(2^(31+l) / d) the quotient is (n*m) >> (31+l)
// (Granlund & Montgomery, "Division by invariant integers using multiplication", Thm 4.2).
struct Magic {
  uint64_t m;
  uint32_t shift;
  uint32_t d;
};

inline Magic make_magic(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned __int128 num = (unsigned __int128)1 << (31 + l);
  uint64_t m = (uint64_t)((num + d - 1) / d);
  return Magic{m, 31 + l, d};
}

__host__ __device__ __forceinline__ uint32_t magic_div(uint32_t n, const Magic& mg) {
  return (uint32_t)(((uint64_t)n * mg.m) >> mg.shift);
}

// Centre of bin index j along an axis, relative to the zero-frequency pixel c, in unbinned
// pixels: b*j + (b-1)/2 - c.  Exact in double (multiples of 1/2 far below 2^53).
__host__ __device__ __forceinline__ double bin_centre(int b, int j, int c) {
  return (double)(b * j - c) + 0.5 * (double)(b - 1);
}

// Kept-bin predicate: centre strictly inside the bright-field disk, |Kc|^2 < r2.
__host__ __device__ __forceinline__ bool bin_kept(double kx, double ky, double r2) {
  return kx * kx + ky * ky < r2;
}

// The kept bins of one bin row form a contiguous run [lo, hi) (a disk meets a line in an
// interval).  Binary searches with the exact predicate.
__host__ __device__ inline void kept_run(int b, int by, int nbx, int cx, int cy, double r2, int& lo,
                                         int& hi) {
  const double ky = bin_centre(b, by, cy);
  // the bin closest to the axis x = 0 (the minimiser of |Kc_x|)
  int best = 0;
  {
    int a = 0, z = nbx - 1;  // last index with centre < 0, if any
    if (bin_centre(b, 0, cx) >= 0.0) {
      best = 0;
    } else {
      while (a < z) {
        int mid = (a + z + 1) / 2;
        if (bin_centre(b, mid, cx) < 0.0) a = mid; else z = mid - 1;
      }
      best = a;
      if (a + 1 < nbx && -bin_centre(b, a, cx) > bin_centre(b, a + 1, cx)) best = a + 1;
    }
  }
  if (!bin_kept(bin_centre(b, best, cx), ky, r2)) {
    lo = hi = 0;
    return;
  }
  int a = 0, z = best;  // first kept in [0, best]
  while (a < z) {
    int mid = (a + z) / 2;
    if (bin_kept(bin_centre(b, mid, cx), ky, r2)) z = mid; else a = mid + 1;
  }
  lo = a;
  a = best;
  z = nbx - 1;  // last kept in [best, nbx)
  while (a < z) {
    int mid = (a + z + 1) / 2;
    if (bin_kept(bin_centre(b, mid, cx), ky, r2)) a = mid; else z = mid - 1;
  }
  hi = a + 1;
}

// Per bin row: first kept pixel number and the run [lo, hi) of kept bx.
struct RowRun {
  int32_t start, lo, hi, pad;
};

}  // namespace stem
