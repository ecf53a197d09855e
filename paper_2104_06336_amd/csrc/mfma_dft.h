// Split-precision scan DFT on the matrix cores (gfx950 v_mfma_f32_32x32x16_{bf16,f16}).
//
// One wavefront transforms a 32 x 32 tile of complex values: B = 1024/N sequences of length
// N = 32 * N2 (the same work unit as the FP32 wave FFT).  With n = N2*a + b (a < 32, b < N2)
// and m = m1 + 32*m2 (m1 < 32, m2 < N2), the DFT of Eq. 2 along one scan axis factors as
//   stage 1   Y[b][m1]  = sum_a x[N2*a + b] W_32^(a*m1)         (32-point DFTs, one MFMA GEMM)
//   twiddle   Y'[b][m1] = Y[b][m1] W_N^(b*m1)                    (FP32, on the MFMA output)
//   stage 2   X[m1 + 32*m2] = sum_b Y'[b][m1] W_N2^(b*m2)        (N2-point DFTs, one MFMA GEMM)
// Rows of the tile are (sequence, b) pairs; stage 2 multiplies by a block-diagonal matrix so
// that sequences do not mix.  Stage 1 takes the data as the A operand (lane l: row l%32,
// k = 8(l/32) + j) and the DFT matrix as B; its result sits with column m1 = l%32 in lane l and
// rows 8(v/4) + 4(l/32) + v%4 in register v.  That result is used directly as the A operand of
// stage 2 (row m1 = l%32; the K order is permuted and the constant B operand is built with the
// same permutation), so no data moves between lanes between the two stages.
//
// Precision: BF16 and FP16 hold only 8 and 11 significant bits.  Each twiddle w is split as
// w = hi + lo with hi = rn(w), lo = rn(w - hi); each non-integer datum likewise.  A product is
// accumulated as hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term, ~2^-16 relative for BF16, is
// dropped).  Event counts below 256 are exact in both formats and are not split.  FP16 has a
// narrow exponent range, so each tile is scaled by a power of two before each stage (the
// largest magnitude lands in [1024, 2048)) and scaled back in FP32 afterwards; both scalings
// are exact.  Twiddles come from the FP32 table of W_1024^t, whose angles are reduced as exact
// integers and evaluated in FP64.
#pragma once

#include "common.h"

namespace stem {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int PREC>
struct SplitTraits;

template <>
struct SplitTraits<STEM_DFT_BF16_SPLIT> {
  using el = __bf16;
  using vec = bf16x8_t;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ f32x16_t mma(vec a, vec b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct SplitTraits<STEM_DFT_FP16_SPLIT> {
  using el = _Float16;
  using vec = f16x8_t;
  static constexpr bool kScaled = true;
  static __device__ __forceinline__ f32x16_t mma(vec a, vec b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// constant operands: 16 per lane (stage, K block, {re hi, re lo, im hi, im lo}), 16 bytes each
constexpr int kMfmaTab = 16 * kWave;

template <typename V>
__device__ __forceinline__ V vneg(V a) {
  uint4 u = __builtin_bit_cast(uint4, a);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(V, u);
}

template <int PREC>
__device__ __forceinline__ void split8(const float* x, typename SplitTraits<PREC>::vec& hi,
                                       typename SplitTraits<PREC>::vec& lo) {
  using E = typename SplitTraits<PREC>::el;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const E h = (E)x[j];
    hi[j] = h;
    lo[j] = (E)(x[j] - (float)h);
  }
}

template <int PREC>
__device__ __forceinline__ typename SplitTraits<PREC>::vec round8(const float* x) {
  using E = typename SplitTraits<PREC>::el;
  typename SplitTraits<PREC>::vec r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = (E)x[j];
  return r;
}

// largest bit pattern of |x| over the wave (non-negative floats order like their bits)
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// power-of-two scale s (and 1/s) that brings the tile's largest magnitude into [1024, 2048)
__device__ __forceinline__ void tile_scale(uint32_t maxbits, float& s, float& inv) {
  int e = (int)((maxbits >> 23) & 0xffu) - 127;
  if (e < -116) e = -116;  // zero or subnormal tile: any scale keeps it representable
  s = __uint_as_float((uint32_t)(127 + 10 - e) << 23);
  inv = __uint_as_float((uint32_t)(127 - 10 + e) << 23);
}

template <int N>
struct MfmaIndex {
  static constexpr int N2 = N / 32;
  // input register i of lane: sequence b, element n
  static __device__ __forceinline__ void in(int lane, int i, int& b, int& n) {
    const int r = lane & 31, h = lane >> 5;
    b = r / N2;
    n = N2 * (16 * (i >> 3) + 8 * h + (i & 7)) + (r % N2);
  }
  // output register i of lane: sequence b, frequency m
  static __device__ __forceinline__ void out(int lane, int i, int& b, int& m) {
    const int c = lane & 31, h = lane >> 5;
    b = c / N2;
    m = 8 * (i >> 2) + 4 * h + (i & 3) + 32 * (c % N2);
  }
};

// Fills the constant operand table (LDS, kMfmaTab entries) from the twiddle table tw[t] = W_1024^t.
template <int N, int PREC>
__device__ __forceinline__ void mfma_fill_table(uint4* tab, const float2* tw, int tid, int nthreads) {
  using E = typename SplitTraits<PREC>::el;
  constexpr int N2 = N / 32;
  for (int e = tid; e < kMfmaTab; e += nthreads) {
    const int o = e / kWave, l = e % kWave;
    const int st = o >> 3, kb = (o >> 2) & 1, part = o & 3;
    const int h = l >> 5, c = l & 31;
    typename SplitTraits<PREC>::vec out;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float2 w;
      if (st == 0) {
        const int a = 16 * kb + 8 * h + j;  // K index of stage 1; column c = m1
        w = tw[((a * c) & 31) * 32];
      } else {
        const int r = 16 * kb + 8 * (j >> 2) + 4 * h + (j & 3);  // stage-1 output row of this K slot
        const int seq = r / N2, b = r % N2, seq_c = c / N2, m2 = c % N2;
        w = seq == seq_c ? tw[((b * m2) % N2) * (1024 / N2)] : make_float2(0.f, 0.f);
      }
      const float x = part < 2 ? w.x : w.y;
      const E hi = (E)x;
      out[j] = (part & 1) ? (E)(x - (float)hi) : hi;
    }
    tab[e] = __builtin_bit_cast(uint4, out);
  }
}

// One K block of a complex product acc += x * F with x split (or exact) and F split.
template <int PREC, bool EXACT>
__device__ __forceinline__ void cmma_block(const float2* x, const uint4* tab, int o0, int lane,
                                           f32x16_t& ar, f32x16_t& ai) {
  using T = SplitTraits<PREC>;
  using V = typename T::vec;
  float xr[8], xi[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xr[j] = x[j].x;
    xi[j] = x[j].y;
  }
  const V frh = __builtin_bit_cast(V, tab[(o0 + 0) * kWave + lane]);
  const V frl = __builtin_bit_cast(V, tab[(o0 + 1) * kWave + lane]);
  const V fih = __builtin_bit_cast(V, tab[(o0 + 2) * kWave + lane]);
  const V fil = __builtin_bit_cast(V, tab[(o0 + 3) * kWave + lane]);
  if constexpr (EXACT) {
    const V rh = round8<PREC>(xr), ih = round8<PREC>(xi);
    const V nih = vneg(ih);
    ar = T::mma(rh, frh, ar);
    ar = T::mma(rh, frl, ar);
    ar = T::mma(nih, fih, ar);
    ar = T::mma(nih, fil, ar);
    ai = T::mma(rh, fih, ai);
    ai = T::mma(rh, fil, ai);
    ai = T::mma(ih, frh, ai);
    ai = T::mma(ih, frl, ai);
  } else {
    V rh, rl, ih, il;
    split8<PREC>(xr, rh, rl);
    split8<PREC>(xi, ih, il);
    const V nih = vneg(ih), nil = vneg(il);
    ar = T::mma(rh, frh, ar);
    ar = T::mma(rh, frl, ar);
    ar = T::mma(rl, frh, ar);
    ar = T::mma(nih, fih, ar);
    ar = T::mma(nih, fil, ar);
    ar = T::mma(nil, fih, ar);
    ai = T::mma(rh, fih, ai);
    ai = T::mma(rh, fil, ai);
    ai = T::mma(rl, fih, ai);
    ai = T::mma(ih, frh, ai);
    ai = T::mma(ih, frl, ai);
    ai = T::mma(il, frh, ai);
  }
}

// Forward DFT of the wave's tile.  v: 16 values per lane in the MfmaIndex::in layout; on
// return the transform in the MfmaIndex::out layout.  EXACT: every input component is an
// integer of magnitude < 256.  tab: table of mfma_fill_table; tw: W_1024^t.
template <int N, int PREC, bool EXACT>
__device__ __forceinline__ void mfma_dft(float2* v, const uint4* tab, const float2* tw, int lane) {
  using T = SplitTraits<PREC>;
  constexpr int N2 = N / 32;
  const int h = lane >> 5, c = lane & 31;
  float inv = 1.f;
  if constexpr (T::kScaled) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      m = max(m, max(__float_as_uint(fabsf(v[i].x)), __float_as_uint(fabsf(v[i].y))));
    float s;
    tile_scale(wave_max_u32(m), s, inv);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_float2(v[i].x * s, v[i].y * s);
  }
  f32x16_t yr, yi;
#pragma unroll
  for (int i = 0; i < 16; ++i) yr[i] = yi[i] = 0.f;
  cmma_block<PREC, EXACT>(v, tab, 0, lane, yr, yi);
  cmma_block<PREC, EXACT>(v + 8, tab, 4, lane, yr, yi);
  // inter-stage twiddle W_N^(b*m1) for row r = (sequence, b) and column m1 = c
  float2 y[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = 8 * (i >> 2) + 4 * h + (i & 3);
    const int b = r % N2;
    const float2 w = tw[b * c * (32 / N2)];
    y[i] = make_float2(yr[i] * w.x - yi[i] * w.y, yr[i] * w.y + yi[i] * w.x);
  }
  if constexpr (T::kScaled) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      m = max(m, max(__float_as_uint(fabsf(y[i].x)), __float_as_uint(fabsf(y[i].y))));
    float s, inv2;
    tile_scale(wave_max_u32(m), s, inv2);
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = make_float2(y[i].x * s, y[i].y * s);
    inv *= inv2;
  }
  f32x16_t gr, gi;
#pragma unroll
  for (int i = 0; i < 16; ++i) gr[i] = gi[i] = 0.f;
  cmma_block<PREC, false>(y, tab, 8, lane, gr, gi);
  cmma_block<PREC, false>(y + 8, tab, 12, lane, gr, gi);
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = make_float2(gr[i] * inv, gi[i] * inv);
}

}  // namespace stem
