// Probe aberration function and the double-overlap predicate (Sec. IV), FP64.
#pragma once

#include "common.h"

namespace stem {

struct Optics {
  double lam, dk, r, r2;
  double c[8];
  double sx, sy;  // detector pixels per scan-frequency index along x and y
  // chi as a polynomial in (wx, wy) = lam*dk*(kx, ky):  p20 wx^2 + p02 wy^2 + p11 wx wy
  //   + p30 wx^3 + p21 wx^2 wy + p12 wx wy^2 + p03 wy^3 + p4 (wx^2 + wy^2)^2
  double lk;
  double p20, p02, p11, p30, p21, p12, p03, p4;
};

// Monomial coefficients of chi (2 pi / lam times the expansion of the eight terms).
inline void optics_poly(Optics& o) {
  const double s = 6.283185307179586476925286766559 / o.lam;
  const double* c = o.c;  // C1, A1a, A1b, B2a, B2b, A2a, A2b, C3
  o.lk = o.lam * o.dk;
  o.p20 = s * (0.5 * c[0] + 0.5 * c[1]);
  o.p02 = s * (0.5 * c[0] - 0.5 * c[1]);
  o.p11 = s * c[2];
  o.p30 = s * (c[3] / 3.0 + c[5] / 3.0);
  o.p21 = s * (c[4] / 3.0 + c[6]);
  o.p12 = s * (c[3] / 3.0 - c[5]);
  o.p03 = s * (c[4] / 3.0 - c[6] / 3.0);
  o.p4 = s * (0.25 * c[7]);
}

__device__ __forceinline__ double chi_poly(double kx_px, double ky_px, const Optics& o) {
  const double wx = kx_px * o.lk, wy = ky_px * o.lk;
  const double xx = wx * wx, yy = wy * wy, w2 = xx + yy;
  return o.p20 * xx + o.p02 * yy + o.p11 * (wx * wy) + xx * (o.p30 * wx + o.p21 * wy) +
         yy * (o.p12 * wx + o.p03 * wy) + o.p4 * (w2 * w2);
}

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

// exp(i psi): psi is reduced in double to r in [-pi/4, pi/4] plus a quadrant (r = psi - q pi/2,
// q an integer), then sin r and cos r are the Taylor polynomials to degree 9 and 10 evaluated in
// float (truncation below 2e-9 on that interval, under float rounding), and the quadrant
// rotates the pair.
__device__ __forceinline__ float2 expi_reduced(double psi) {
  const double two_pi = 6.283185307179586476925286766559;
  const double inv_two_pi = 0.15915494309189533576888376337251;
  const double half_pi = 1.5707963267948966192313216916398;
  const double two_over_pi = 0.63661977236758134307553505349006;
  const double red = psi - two_pi * rint(psi * inv_two_pi);  // [-pi, pi]
  const double qd = rint(red * two_over_pi);                  // -2 .. 2
  const float x = (float)(red - qd * half_pi);
  const float x2 = x * x;
  const float sn = x * (1.f + x2 * (-1.f / 6.f + x2 * (1.f / 120.f + x2 * (-1.f / 5040.f + x2 * (1.f / 362880.f)))));
  const float cs = 1.f + x2 * (-0.5f + x2 * (1.f / 24.f + x2 * (-1.f / 720.f + x2 * (1.f / 40320.f +
                                                                               x2 * (-1.f / 3628800.f)))));
  switch ((int)qd & 3) {
    case 0: return make_float2(cs, sn);
    case 1: return make_float2(-sn, cs);
    case 2: return make_float2(-cs, -sn);
    default: return make_float2(sn, -cs);
  }
}

}  // namespace stem
