// Mixed-radix FFT of any length N = 2^a 3^b 5^c up to kGenMax, for the scan sizes the wavefront FFT
// of fft_wave.h does not take (not a power of two, or longer than 1024).
//
// A workgroup transforms RB = max(1, 4096/N) rows at once in LDS with a Stockham autosort FFT:
// pass s of radix R, with Ns the product of the earlier radices, takes butterfly j (0 <= j < N/R)
// from elements j + q N/R (q < R), multiplies element q by w^(q (j mod Ns)) with w =
// exp(-2 pi i / (Ns R)), applies the length-R DFT and writes element q to
// (j div Ns) Ns R + (j mod Ns) + q Ns.  Every thread reads all its butterflies' inputs before the
// workgroup barrier and writes after it, so one LDS buffer serves each pass in place.  Twiddles
// come from an LDS table of W_N^t = exp(-2 pi i t/N), t < N, evaluated in FP64 with the angle
// 2t/N (an exact integer ratio) and rounded to FP32; the exponent q (j mod Ns) N/(Ns R) is an
// integer below N.  Radices are taken as 4 while 4 divides what is left, then 2, 3, 5.
#pragma once

#include "common.h"

namespace stem {

constexpr int kGenMax = 4096;     // longest transform
constexpr int kGenThreads = 256;  // threads of a generic-FFT workgroup
constexpr int kGenMaxPasses = 12;

struct GPlan {
  int32_t n;
  int32_t np;
  int32_t r[kGenMaxPasses];
};

// N = 2^a 3^b 5^c with 2 <= N <= kGenMax, factored into passes; false otherwise.
inline bool gen_plan(int n, GPlan& p) {
  if (n < 2 || n > kGenMax) return false;
  p.n = n;
  p.np = 0;
  int m = n;
  while (m % 4 == 0 && p.np < kGenMaxPasses) { p.r[p.np++] = 4; m /= 4; }
  while (m % 2 == 0 && p.np < kGenMaxPasses) { p.r[p.np++] = 2; m /= 2; }
  while (m % 3 == 0 && p.np < kGenMaxPasses) { p.r[p.np++] = 3; m /= 3; }
  while (m % 5 == 0 && p.np < kGenMaxPasses) { p.r[p.np++] = 5; m /= 5; }
  return m == 1;
}

__host__ __device__ inline int gen_rows_per_block(int n) { return n >= kGenMax ? 1 : kGenMax / n; }

// tw[t] = exp(-2 pi i t / n), t < n (FP64 evaluation, FP32 rounding); every thread of the workgroup
// takes part
__device__ __forceinline__ void gen_twiddles(float2* tw, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    tw[t] = make_float2((float)c, (float)-s);
  }
}

// length-R DFTs in registers (forward sign), natural order in and out
__device__ __forceinline__ void gdft2(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void gdft4(float2* v) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, cmul_mi(t3));
  v[3] = csub(t1, cmul_mi(t3));
}

// X_k = sum_n x_n exp(-2 pi i n k / 3): with s = x1 + x2, d = x1 - x2,
// X_0 = x0 + s, X_{1,2} = x0 - s/2 -/+ i (sqrt(3)/2) d
__device__ __forceinline__ void gdft3(float2* v) {
  constexpr float h = 0.86602540378443864676f;  // sqrt(3)/2
  const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
  const float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
  const float2 r = make_float2(h * d.y, -h * d.x);  // -i (sqrt(3)/2) d
  v[0] = cadd(v[0], s);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

// length 5 from its definition, with cos and sin of 2 pi/5 and 4 pi/5: pairs (x1, x4) and (x2, x3)
// give X_k = x0 + c_k1 (x1 + x4) + c_k2 (x2 + x3) - i (s_k1 (x1 - x4) + s_k2 (x2 - x3))
__device__ __forceinline__ void gdft5(float2* v) {
  constexpr float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;  // cos 2pi/5, cos 4pi/5
  constexpr float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;   // sin 2pi/5, sin 4pi/5
  const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  const float2 x0 = v[0];
  const float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  const float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  const float2 q1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);   // k = 1
  const float2 q2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);   // k = 2
  v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = make_float2(p1.x + q1.y, p1.y - q1.x);  // p1 - i q1
  v[4] = make_float2(p1.x - q1.y, p1.y + q1.x);  // p1 + i q1
  v[2] = make_float2(p2.x + q2.y, p2.y - q2.x);
  v[3] = make_float2(p2.x - q2.y, p2.y + q2.x);
}

// One Stockham pass of radix R over rb rows of length n at buf[row * n + i] (blockDim.x ==
// kGenThreads).  The twiddle exponent q (j mod Ns) n/(Ns R) is below n.
template <int R>
__device__ __forceinline__ void gen_pass(float2* buf, const float2* tw, int n, int rb, int ns) {
  const int m = n / R;               // butterflies per row
  const int tstride = n / (ns * R);  // twiddle index step of exponent 1
  const int total = rb * m;
  // butterflies per thread: rb n <= kGenMax elements make at most kGenMax / R butterflies
  constexpr int kMaxB = (kGenMax / R + kGenThreads - 1) / kGenThreads;
  float2 v[kMaxB][R];
#pragma unroll
  for (int b = 0; b < kMaxB; ++b) {
    const int g = threadIdx.x + b * kGenThreads;
    if (g < total) {
      const int row = g / m, j = g % m;
      const float2* in = buf + row * n;
      const int k = j % ns;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        float2 x = in[j + q * m];
        if (q > 0 && ns > 1) x = cmul(x, tw[q * k * tstride]);
        v[b][q] = x;
      }
      if constexpr (R == 2) gdft2(v[b]);
      else if constexpr (R == 3) gdft3(v[b]);
      else if constexpr (R == 4) gdft4(v[b]);
      else gdft5(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kMaxB; ++b) {
    const int g = threadIdx.x + b * kGenThreads;
    if (g < total) {
      const int row = g / m, j = g % m;
      float2* out = buf + row * n;
      const int base = (j / ns) * ns * R + (j % ns);
#pragma unroll
      for (int q = 0; q < R; ++q) out[base + q * ns] = v[b][q];
    }
  }
  __syncthreads();
}

// Forward FFT of rb rows of length p.n in buf (LDS), in place; tw from gen_twiddles.
__device__ __forceinline__ void gen_fft(float2* buf, const float2* tw, const GPlan& p, int rb) {
  int ns = 1;
  for (int s = 0; s < p.np; ++s) {
    const int r = p.r[s];
    if (r == 4) gen_pass<4>(buf, tw, p.n, rb, ns);
    else if (r == 2) gen_pass<2>(buf, tw, p.n, rb, ns);
    else if (r == 3) gen_pass<3>(buf, tw, p.n, rb, ns);
    else gen_pass<5>(buf, tw, p.n, rb, ns);
    ns *= r;
  }
}

}  // namespace stem
