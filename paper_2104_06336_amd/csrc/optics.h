// Probe aberration function and the double-overlap predicate (Sec. IV), FP64.
#pragma once

#include "common.h"

namespace stem {

struct Optics {
  double lam, dk, r, r2;
  double c[8];
  double sx, sy;  // detector pixels per scan-frequency index along x and y
};

// d chi / d c_j at a detector coordinate given in unbinned pixels (j = C1, A1a, A1b, B2a, B2b,
// A2a, A2b, C3); chi = sum_j c_j B_j.
__device__ __forceinline__ void chi_basis(double kx_px, double ky_px, const Optics& o, double* bj) {
  const double wx = o.lam * (kx_px * o.dk);
  const double wy = o.lam * (ky_px * o.dk);
  const double wxx = wx * wx, wyy = wy * wy, w2 = wxx + wyy;
  const double s = 6.283185307179586476925286766559 / o.lam;
  const double third = 1.0 / 3.0;
  bj[0] = s * (0.5 * w2);
  bj[1] = s * (0.5 * (wxx - wyy));
  bj[2] = s * (wx * wy);
  bj[3] = s * (third * w2 * wx);
  bj[4] = s * (third * w2 * wy);
  bj[5] = s * (third * (wxx * wx - 3.0 * wx * wyy));
  bj[6] = s * (third * (3.0 * wxx * wy - wyy * wy));
  bj[7] = s * (0.25 * w2 * w2);
}

__device__ __forceinline__ double chi_px(double kx_px, double ky_px, const Optics& o) {
  double b[8];
  chi_basis(kx_px, ky_px, o, b);
  double x = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) x += o.c[j] * b[j];
  return x;
}

// Signed scan-frequency index (numpy fftfreq order: n/2 -> -n/2).
__device__ __forceinline__ int signed_index(int m, int n) { return m < (n + 1) / 2 ? m : m - n; }

// Double-overlap membership of pixel K for frequency Q: |K| < r, |K - Q| < r, |K + Q| >= r,
// every operation rounded separately (no fused multiply-add), as the reference evaluation.
__device__ __forceinline__ bool double_overlap(double kx, double ky, double qx, double qy, double r2) {
#pragma clang fp contract(off)
  const double k2 = kx * kx + ky * ky;
  const double dx = kx - qx, dy = ky - qy;
  const double d2 = dx * dx + dy * dy;
  const double ux = kx + qx, uy = ky + qy;
  const double u2 = ux * ux + uy * uy;
  return (k2 < r2) && (d2 < r2) && (u2 >= r2);
}

// exp(i psi) with psi reduced to [-pi, pi] in double, then evaluated in float.
__device__ __forceinline__ float2 expi_reduced(double psi) {
  const double inv2pi = 0.15915494309189533576888376337251;
  const double two_pi = 6.283185307179586476925286766559;
  const double red = psi - two_pi * rint(psi * inv2pi);
  float s, c;
  sincosf((float)red, &s, &c);
  return make_float2(c, s);
}

}  // namespace stem
