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
  // float screening of the double-overlap test: thresholds r2 -/+ a bound on the float error
  float sxf, syf, r2lo, r2hi;
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

// Thresholds of the float screening.  With |K| <= r, |Q| <= qmax and M = r + qmax, the float
// evaluation of (Kx -/+ Qx)^2 + (Ky -/+ Qy)^2 (K rounded once to float, Q = i * float(s) rounded
// twice, then the difference, the squares and the sum) differs from the exact value by less than
// 20 eps M^2 (eps = 2^-24); the margin is 32 eps M^2 plus 8 eps r^2 for the rounding of the
// thresholds themselves, so a float result outside [r2lo, r2hi] decides the double test.
inline void optics_screen(Optics& o, int ny, int nx) {
  const double eps = 1.0 / 16777216.0;
  const double qx = 0.5 * nx * o.sx, qy = 0.5 * ny * o.sy;
  const double M = o.r + __builtin_sqrt(qx * qx + qy * qy);
  const double margin = 32.0 * eps * M * M + 8.0 * eps * o.r2 + 1e-30;
  o.sxf = (float)o.sx;
  o.syf = (float)o.sy;
  o.r2lo = (float)(o.r2 - margin);
  o.r2hi = (float)(o.r2 + margin);
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

// Double-overlap membership of a kept pixel K (|K| < r holds for every kept pixel by the same
// predicate) for the frequency with signed indices (ix, iy): decided in float when both float
// distances clear r^2 by the error margin, otherwise by the reference double evaluation.
__device__ __forceinline__ bool overlap_screened(double kx, double ky, float kxf, float kyf, int ix, int iy,
                                                 const Optics& o) {
  const float qxf = (float)ix * o.sxf, qyf = (float)iy * o.syf;
  const float dx = kxf - qxf, dy = kyf - qyf;
  const float d2 = dx * dx + dy * dy;
  const float ux = kxf + qxf, uy = kyf + qyf;
  const float u2 = ux * ux + uy * uy;
  if (d2 > o.r2hi || u2 < o.r2lo) return false;
  if (d2 < o.r2lo && u2 > o.r2hi) return true;
  return double_overlap(kx, ky, (double)ix * o.sx, (double)iy * o.sy, o.r2);
}

// ---------------------------------------------------------------------------------------------
// The double-overlap set of one pixel K along one scan-frequency column.  For a fixed column
// (fixed Qx, signed index ix) and Qy = iy*sy increasing with iy, the rounded distance
// fl(fl(dx^2) + fl(dy^2)) with dy = fl(Ky - Qy) is non-increasing and then non-decreasing in iy
// (IEEE rounding is monotone), so {iy : |K - Q|^2 < r^2} is one interval [a0, a1] and
// {iy : |K + Q|^2 < r^2} another, [b0, b1]; the set is [a0, a1] minus [b0, b1] (|K| < r holds
// for every kept pixel).  The bounds come from a square-root estimate corrected by the exact
// double test of `double_overlap`, so membership equals that test for every iy.

// |K - Q|^2 < r^2 (sgn = -1) or |K + Q|^2 < r^2 (sgn = +1), evaluated as the reference does
__device__ __forceinline__ bool near_disk(double kx, double ky, double qx, double qy, double r2, int sgn) {
#pragma clang fp contract(off)
  const double dx = sgn < 0 ? kx - qx : kx + qx;
  const double dy = sgn < 0 ? ky - qy : ky + qy;
  return dx * dx + dy * dy < r2;
}

// Interval of iy in [lo, hi] (inclusive) where near_disk holds along the column Qx = qx; empty
// when lo_out > hi_out.  ny: number of frequencies (iy in [-ny/2, ny/2)).
__device__ __forceinline__ void disk_interval(double kx, double ky, double qx, double sy, double r, double r2, int sgn,
                                              int ny, int& lo_out, int& hi_out) {
  const int imin = -ny / 2, imax = ny / 2 - 1;
  // centre: Qy = -sgn*... (K - Q: Qy = Ky; K + Q: Qy = -Ky)
  const double cy = sgn < 0 ? ky : -ky;
  const double dxv = sgn < 0 ? kx - qx : kx + qx;
  const double h2 = r2 - dxv * dxv;
  lo_out = 1;
  hi_out = 0;
  if (!(h2 > -1e-9 * r2)) return;  // |dx| well beyond r: empty (the exact test is checked at the centre)
  const double h = sqrt(h2 > 0.0 ? h2 : 0.0);
  int c0 = (int)floor(cy / sy);
  if (c0 < imin) c0 = imin;
  if (c0 > imax) c0 = imax;
  // the minimum of the V lies at c0 or a neighbour (c0 = floor(cy/sy) may be off by one after
  // rounding); if the test fails at all three the set is empty
  int c = c0;
  if (!near_disk(kx, ky, qx, (double)c * sy, r2, sgn)) {
    c = c0 + 1;
    if (c > imax || !near_disk(kx, ky, qx, (double)c * sy, r2, sgn)) {
      c = c0 - 1;
      if (c < imin || !near_disk(kx, ky, qx, (double)c * sy, r2, sgn)) return;
    }
  }
  // upper end: estimate, then walk to the exact boundary
  int u = (int)floor((cy + h) / sy);
  if (u < c) u = c;
  if (u > imax) u = imax;
  while (u > c && !near_disk(kx, ky, qx, (double)u * sy, r2, sgn)) --u;
  while (u < imax && near_disk(kx, ky, qx, (double)(u + 1) * sy, r2, sgn)) ++u;
  int l = (int)ceil((cy - h) / sy);
  if (l > c) l = c;
  if (l < imin) l = imin;
  while (l < c && !near_disk(kx, ky, qx, (double)l * sy, r2, sgn)) ++l;
  while (l > imin && near_disk(kx, ky, qx, (double)(l - 1) * sy, r2, sgn)) --l;
  lo_out = l;
  hi_out = u;
}

// chi along one column as a polynomial in wy = lam*dk*(Ky - Qy) for fixed wx = lam*dk*(Kx - Qx):
// chi = h0 + wy (h1 + wy (h2 + wy (h3 + wy h4)))
struct ChiCol {
  double h0, h1, h2, h3, h4;
};

__device__ __forceinline__ ChiCol chi_column(double wx, const Optics& o) {
  const double xx = wx * wx;
  ChiCol c;
  c.h0 = xx * (o.p20 + wx * o.p30 + xx * o.p4);
  c.h1 = wx * (o.p11 + wx * o.p21);
  c.h2 = o.p02 + wx * o.p12 + 2.0 * o.p4 * xx;
  c.h3 = o.p03;
  c.h4 = o.p4;
  return c;
}

__device__ __forceinline__ double chi_eval(const ChiCol& c, double wy) {
  return c.h0 + wy * (c.h1 + wy * (c.h2 + wy * (c.h3 + wy * c.h4)));
}

// chi(K - Q) - chi(Kc) - theta along one column as a polynomial in the signed row index iy, in
// revolutions (divided by 2 pi): with wy = A + B iy (A = lam dk Ky, B = -lam dk sy), the quartic of
// chi_column expanded in powers of iy, the constant term less kch.
// psi / (2 pi) = p0 + iy (p1 + iy (p2 + iy (p3 + iy p4))).
struct ChiRow {
  double p0, p1, p2, p3, p4;
};

__device__ __forceinline__ ChiRow chi_row(const ChiCol& c, double A, double B, double kch) {
  const double inv_two_pi = 0.15915494309189533576888376337251;
  const double A2 = A * A, A3 = A2 * A, A4 = A2 * A2;
  const double B2 = B * B, B3 = B2 * B, B4 = B2 * B2;
  ChiRow r;
  r.p0 = ((c.h0 + A * c.h1 + A2 * c.h2 + A3 * c.h3 + A4 * c.h4) - kch) * inv_two_pi;
  r.p1 = B * (c.h1 + 2.0 * A * c.h2 + 3.0 * A2 * c.h3 + 4.0 * A3 * c.h4) * inv_two_pi;
  r.p2 = B2 * (c.h2 + 3.0 * A * c.h3 + 6.0 * A2 * c.h4) * inv_two_pi;
  r.p3 = B3 * (c.h3 + 4.0 * A * c.h4) * inv_two_pi;
  r.p4 = B4 * c.h4 * inv_two_pi;
  return r;
}

__device__ __forceinline__ double chi_row_eval(const ChiRow& r, double t) {
  return r.p0 + t * (r.p1 + t * (r.p2 + t * (r.p3 + t * r.p4)));
}

// exp(2 pi i r) for a phase r in revolutions: r is reduced in FP64 to f = r - rint(r) in
// [-1/2, 1/2], rounded to float; the hardware sine and cosine of 2 pi f (v_sin_f32 / v_cos_f32,
// whose argument is in revolutions) give the pair.
__device__ __forceinline__ float2 expi_rev(double r) {
  const float f = (float)(r - rint(r));
  return make_float2(__builtin_amdgcn_cosf(f), __builtin_amdgcn_sinf(f));
}

// exp(i psi): psi / (2 pi) (error below |psi / 2 pi| ulp(1/(2 pi)) + ulp) through expi_rev.
__device__ __forceinline__ float2 expi_reduced(double psi) {
  const double inv_two_pi = 0.15915494309189533576888376337251;
  return expi_rev(psi * inv_two_pi);
}

// Double-overlap sets of pixel K along column ix: iy in [a0, a1] but not in [b0, b1].
struct ColSet {
  int a0, a1, b0, b1;
  __device__ __forceinline__ bool has(int iy) const { return iy >= a0 && iy <= a1 && !(iy >= b0 && iy <= b1); }
  __device__ __forceinline__ bool empty() const { return a0 > a1; }
};

__device__ __forceinline__ ColSet col_set(double kx, double ky, int ix, int ny, const Optics& o) {
  const double qx = (double)ix * o.sx;
  ColSet cs;
  disk_interval(kx, ky, qx, o.sy, o.r, o.r2, -1, ny, cs.a0, cs.a1);
  if (cs.a0 > cs.a1) {
    cs.b0 = 1;
    cs.b1 = 0;
    return cs;
  }
  disk_interval(kx, ky, qx, o.sy, o.r, o.r2, +1, ny, cs.b0, cs.b1);
  return cs;
}

// The double-overlap interval table of the fused column sum and its active-pixel mask: for
// column set cs (B consecutive half-spectrum columns, colset_width) and mask word w, lane j takes
// pixel kd = 64 w + j; cst[kd * nc + c] packs its direct and mirrored sets of every column c of
// the set, and bit j of mask[cs * nmw + w] says whether any of them is non-empty.
struct SetsJob {
  Optics o;
  int n_k, nx, ny, ncs, nmw;
  int4* cst;          // nullptr: nothing to do
  uint64_t* mask;
  int B;              // half-spectrum columns per column set
};

// Half-spectrum columns per column set: the B = 1024/Ny columns one wave of the fused kernels takes
// (one column for the lengths those kernels do not take).
__host__ __device__ inline int colset_width(int ny) { return (ny >= 32 && ny <= 1024 && (ny & (ny - 1)) == 0) ? 1024 / ny : 1; }

// One mask word (one wave, every lane active); k = Kc of the lane's pixel when kd < n_k.
__device__ __forceinline__ void sets_word(const SetsJob& j, int64_t word, int lane, double2 k) {
  const int nc = j.nx / 2 + 1, B = j.B;
  const int cs = (int)(word / j.nmw), w = (int)(word % j.nmw);
  const int kd = 64 * w + lane;
  auto pk = [](int lo, int hi) { return (int)(((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16)); };
  bool any = false;
  if (kd < j.n_k) {
    const int c1 = cs * B + B < nc ? cs * B + B : nc;
    for (int c = cs * B; c < c1; ++c) {
      const ColSet d = col_set(k.x, k.y, signed_index(c, j.nx), j.ny, j.o);
      ColSet m{1, 0, 1, 0};
      if (c > 0 && 2 * c < j.nx) m = col_set(k.x, k.y, signed_index(j.nx - c, j.nx), j.ny, j.o);
      j.cst[(int64_t)kd * nc + c] = make_int4(pk(d.a0, d.a1), pk(d.b0, d.b1), pk(m.a0, m.a1), pk(m.b0, m.b1));
      any = any || d.a0 <= d.a1 || m.a0 <= m.a1;
    }
  }
  const uint64_t bits = __ballot(any);
  if (lane == 0) j.mask[word] = bits;
}

}  // namespace stem
