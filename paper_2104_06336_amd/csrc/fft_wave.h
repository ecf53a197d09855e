// Wavefront-level FFT for power-of-two lengths N = 32 ... 1024 on gfx950.
//
// One wave (64 lanes) transforms B = 1024/N independent length-N sequences at once; every
// lane holds 16 complex values in registers.  The transform is a Stockham autosort FFT
// (mixed radix: 16, 16, then 2/4/8 as needed; at most three passes); between passes the
// data goes through a wave-private LDS buffer of 1024 (+64 padding) float2.  In pass s with
// radix R and Ns = product of earlier radices, butterfly j of a sequence reads elements
// j + r*N/R (r < R), multiplies element r by w^(r*(j mod Ns)) with w = exp(-2 pi i/(Ns R)),
// applies a length-R DFT and writes element r to (j div Ns)*Ns*R + (j mod Ns) + r*Ns.
//
// Register layout (index i in [0, 16)) -- the caller loads inputs and stores outputs in it:
//   input  : sequence b = lane / (N/16), element (lane % (N/16)) + i*(N/16)
//   output : with Rl the last radix, butterfly g = lane + 64*(i / Rl), r = i % Rl,
//            sequence b = g / (N/Rl), element (g % (N/Rl)) + r*(N/Rl)
// Forward direction (exp(-2 pi i ...)); the inverse is obtained by conjugating in and out.
#pragma once

#include "common.h"

namespace stem {

constexpr int kFftLds = 1024 + 64;  // float2 per wave

// tw[t] = exp(-2 pi i t / 1024), FP32 rounded from an FP64 evaluation with exact angle t/512.
__device__ __forceinline__ void fill_twiddles(float2* tw, int tid, int nthreads) {
  // Only the first octant is evaluated: (cos, sin)(pi u / 512) for u = 0 .. 128 from FP64
  // sincospi, rounded to FP32.  With t = 256 q + r, the angle pi t / 512 is q quarter turns plus
  // phi = pi r / 512, and phi is pi u / 512 (r <= 128) or pi/2 - pi u / 512 (u = 256 - r), so every
  // entry is a sign change or swap of an octant value: exact, and equal to the rounded value
  // itself.  Every thread of the workgroup takes part (the function synchronises it); nthreads >= 64.
  for (int u = tid; u <= 128; u += nthreads) {
    double s, c;
    sincospi((double)u / 512.0, &s, &c);
    tw[u] = make_float2((float)c, (float)s);
  }
  __syncthreads();
  float2 val[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int t = tid + k * nthreads;
    if (t < 1024) {
      const int q = t >> 8, r = t & 255;
      const float2 o = tw[r <= 128 ? r : 256 - r];
      const float cp = r <= 128 ? o.x : o.y, sp = r <= 128 ? o.y : o.x;  // cos, sin of phi
      float c, sn;
      if (q == 0) { c = cp; sn = sp; }
      else if (q == 1) { c = -sp; sn = cp; }
      else if (q == 2) { c = -cp; sn = -sp; }
      else { c = sp; sn = -cp; }
      val[k] = make_float2(c, -sn);  // exp(-i pi t / 512)
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int t = tid + k * nthreads;
    if (t < 1024) tw[t] = val[k];
  }
}

__device__ __forceinline__ int fft_pad(int i) { return i + (i >> 4); }

// Orders LDS traffic of one wavefront (all lanes) across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------------------------
// small DFTs in registers, natural-order in and out, forward sign

__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, cmul_mi(t3));
  a3 = csub(t1, cmul_mi(t3));
}

__device__ __forceinline__ void dft4(float2* v) { dft4(v[0], v[1], v[2], v[3]); }

// exp(-2 pi i m / 16), m = 0..15
__device__ __forceinline__ float2 w16(int m) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, h = 0.70710678118654752f;
  switch (m & 15) {
    case 0: return make_float2(1.f, 0.f);
    case 1: return make_float2(c1, -s1);
    case 2: return make_float2(h, -h);
    case 3: return make_float2(s1, -c1);
    case 4: return make_float2(0.f, -1.f);
    case 5: return make_float2(-s1, -c1);
    case 6: return make_float2(-h, -h);
    case 7: return make_float2(-c1, -s1);
    case 8: return make_float2(-1.f, 0.f);
    case 9: return make_float2(-c1, s1);
    case 10: return make_float2(-h, h);
    case 11: return make_float2(-s1, c1);
    case 12: return make_float2(0.f, 1.f);
    case 13: return make_float2(s1, c1);
    case 14: return make_float2(h, h);
    default: return make_float2(c1, s1);
  }
}

// length 8 = 2 x 4 (n = n1 + 2 n2, X[k2 + 4 k1])
__device__ __forceinline__ void dft8(float2* v) {
  float2 y[2][4];
#pragma unroll
  for (int n1 = 0; n1 < 2; ++n1) {
    y[n1][0] = v[n1];
    y[n1][1] = v[n1 + 2];
    y[n1][2] = v[n1 + 4];
    y[n1][3] = v[n1 + 6];
    dft4(y[n1]);
  }
#pragma unroll
  for (int k2 = 1; k2 < 4; ++k2) y[1][k2] = cmul(y[1][k2], w16(2 * k2));
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    v[k2] = cadd(y[0][k2], y[1][k2]);
    v[k2 + 4] = csub(y[0][k2], y[1][k2]);
  }
}

// length 16 = 4 x 4 (n = n1 + 4 n2, X[k2 + 4 k1])
__device__ __forceinline__ void dft16(float2* v) {
  float2 y[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    y[n1][0] = v[n1];
    y[n1][1] = v[n1 + 4];
    y[n1][2] = v[n1 + 8];
    y[n1][3] = v[n1 + 12];
    dft4(y[n1]);
  }
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) y[n1][k2] = cmul(y[n1][k2], w16(n1 * k2));
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 a0 = y[0][k2], a1 = y[1][k2], a2 = y[2][k2], a3 = y[3][k2];
    dft4(a0, a1, a2, a3);
    v[k2] = a0;
    v[k2 + 4] = a1;
    v[k2 + 8] = a2;
    v[k2 + 12] = a3;
  }
}

template <int R>
__device__ __forceinline__ void dft_r(float2* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v);
  else if constexpr (R == 8) dft8(v);
  else dft16(v);
}

// ---------------------------------------------------------------------------------------------
// plans

template <int N> struct FftPlan;
template <> struct FftPlan<1024> { static constexpr int P = 3, R0 = 16, R1 = 16, R2 = 4; };
template <> struct FftPlan<512> { static constexpr int P = 3, R0 = 16, R1 = 16, R2 = 2; };
template <> struct FftPlan<256> { static constexpr int P = 2, R0 = 16, R1 = 16, R2 = 1; };
template <> struct FftPlan<128> { static constexpr int P = 2, R0 = 16, R1 = 8, R2 = 1; };
template <> struct FftPlan<64> { static constexpr int P = 2, R0 = 16, R1 = 4, R2 = 1; };
template <> struct FftPlan<32> { static constexpr int P = 2, R0 = 16, R1 = 2, R2 = 1; };

template <int N> constexpr int fft_last_radix() {
  return FftPlan<N>::P == 3 ? FftPlan<N>::R2 : FftPlan<N>::R1;
}

// One Stockham pass.  FIRST: inputs already in registers.  LAST: outputs stay in registers.
template <int N, int R, int NS, bool FIRST, bool LAST>
__device__ __forceinline__ void fft_pass(float2* v, float2* lds, const float2* tw, int lane) {
  constexpr int NB = N / R;  // butterflies per sequence
  constexpr int Q = 16 / R;  // butterflies per lane
  if constexpr (!FIRST) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int g = lane + kWave * q;
      const int b = g / NB, j = g % NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q * R + r] = lds[fft_pad(b * N + j + r * NB)];
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if constexpr (NS > 1) {
      const int j = (lane + kWave * q) % NB;
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[q * R + r] = cmul(v[q * R + r], tw[r * k * (1024 / (NS * R))]);
    }
    dft_r<R>(v + q * R);
  }
  if constexpr (!LAST) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int g = lane + kWave * q;
      const int b = g / NB, j = g % NB;
      const int base = b * N + (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[fft_pad(base + r * NS)] = v[q * R + r];
    }
    wave_lds_sync();
  }
}

// Forward FFT of B = 1024/N sequences held as described at the top of this file.
// lds: wave-private buffer of kFftLds float2; tw: the 1024-entry twiddle table (LDS).
template <int N>
__device__ __forceinline__ void wave_fft(float2* v, float2* lds, const float2* tw, int lane) {
  using P = FftPlan<N>;
  if constexpr (P::P == 2) {
    fft_pass<N, P::R0, 1, true, false>(v, lds, tw, lane);
    fft_pass<N, P::R1, P::R0, false, true>(v, lds, tw, lane);
  } else {
    fft_pass<N, P::R0, 1, true, false>(v, lds, tw, lane);
    fft_pass<N, P::R1, P::R0, false, false>(v, lds, tw, lane);
    fft_pass<N, P::R2, P::R0 * P::R1, false, true>(v, lds, tw, lane);
  }
}

// Index maps of the register layout.
template <int N>
__device__ __forceinline__ void fft_in_index(int lane, int i, int& b, int& n) {
  constexpr int NB = N / 16;
  b = lane / NB;
  n = lane % NB + i * NB;
}

template <int N>
__device__ __forceinline__ void fft_out_index(int lane, int i, int& b, int& n) {
  constexpr int RL = fft_last_radix<N>();
  constexpr int NB = N / RL;
  const int g = lane + kWave * (i / RL);
  b = g / NB;
  n = g % NB + (i % RL) * NB;
}

}  // namespace stem
