// Batched row FFTs (power-of-two lengths 32..1024) and the centre-of-mass DPC path
// (Eq. 4 and the regularised Fourier gradient descent of Sec. V).
//
// k_row_fft: a workgroup of W = 8 waves (4 when there are too few rows to give every CU a
// workgroup); each wave transforms B = 1024/N rows at a time with the wavefront FFT of
// fft_wave.h.  Row-major outputs are stored straight from registers; transposed outputs
// (element (r, m) -> out[m*stride + r]) are first staged in the waves' LDS buffers so that the
// workgroup writes runs of W B consecutive rows per frequency.
#include <mutex>

#include "common.h"
#include "fft_generic.h"
#include "fft_wave.h"
#include "kernels.h"
#include "trace.h"

namespace stem {

constexpr int kWaveStride = kFftLds + 4;  // float2 per wave buffer; the +4 staggers LDS banks

// SUM: the input is the sum of a.nparts partial planes (in_mode IN_C64_SUM), read four at a time;
// a separate instantiation, so that the other input modes keep their lower register count.  SEG
// (with SUM): the partials are segments, row r adding rows a.part_seg[r] .. a.part_seg[r+1]-1.
template <int N, bool INV, int W, bool SUM, bool SEG = false>
__global__ void __launch_bounds__(64 * W) k_row_fft(RowFftArgs a, int in_mode, int out_mode) {
  constexpr int kRowThreads = 64 * W;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[W * kWaveStride];
  constexpr int B = 1024 / N;
  constexpr int TR = W * B;  // rows per tile
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if constexpr (SUM) {
    if (a.stats && blockIdx.x == 0) {
      // every thread of the first workgroup sums a strided share, four loads in flight
      // per wave: pair count below bit 40, 8-byte loads above
      __shared__ unsigned long long s_red[2][W];
      constexpr unsigned long long kLow = (1ull << 40) - 1;
      unsigned long long c0 = 0, c1 = 0, l0 = 0, l1 = 0;
      for (int64_t i = threadIdx.x; i < a.nwcnt; i += 2 * kRowThreads) {
        const unsigned long long u = a.wcnt[i];
        c0 += u & kLow;
        l0 += u >> 40;
        if (i + kRowThreads < a.nwcnt) {
          const unsigned long long v = a.wcnt[i + kRowThreads];
          c1 += v & kLow;
          l1 += v >> 40;
        }
      }
      unsigned long long c = c0 + c1, l = l0 + l1;
      for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off);
        l += __shfl_xor(l, off);
      }
      if (lane == 0) {
        s_red[0][wave] = c;
        s_red[1][wave] = l;
      }
      __syncthreads();
      if (threadIdx.x < 4) {
        unsigned long long t = 0, u = 0;
        for (int w = 0; w < W; ++w) {
          t += s_red[0][w];
          u += s_red[1][w];
        }
        a.stats[threadIdx.x] = threadIdx.x == 0   ? t
                               : threadIdx.x == 1 ? (a.part_seg ? (unsigned long long)a.part_seg[a.nrows]
                                                                : (unsigned long long)a.stats_groups)
                               : threadIdx.x == 2 ? 8ull * u
                                                  : (unsigned long long)a.stats_chunks;
      }
      if (threadIdx.x == 4 && a.ready_out) *a.ready_out = a.ready_val;
    }
  }
  fill_twiddles(s_tw, threadIdx.x, kRowThreads);
  __syncthreads();
  float2* buf = s_buf + wave * kWaveStride;
  const int64_t ntiles = (a.nrows + TR - 1) / TR;
  const bool transposed = out_mode == OUT_T_C64 || out_mode == OUT_T_RE || out_mode == OUT_T_IM;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TR + wave * B;
    float2 v[16];
    if constexpr (SUM) {
      // partial sums added in a fixed order; the 64 loads of four partials are issued together
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = make_float2(0.f, 0.f);
      auto load_part = [&](int p, float2* t) {
        const float2* src = a.in_c + (int64_t)p * a.part_stride;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          int b, n;
          fft_in_index<N>(lane, i, b, n);
          const int64_t r = r0 + b;
          t[i] = r < a.nrows ? src[r * N + n] : make_float2(0.f, 0.f);
        }
      };
      if constexpr (SEG) {
        // segments: row r adds rows part_seg[r] .. part_seg[r + 1] - 1, in order (a lane's 16
        // elements are of one row); the wave runs to the largest count among its rows
        int b, n;
        fft_in_index<N>(lane, 0, b, n);
        const int64_t r = r0 + b;
        const int64_t s0 = r < a.nrows ? min(max(a.part_seg[r], (int64_t)0), a.part_seg_rows) : 0;
        const int sn = r < a.nrows ? (int)(min(max(a.part_seg[r + 1], s0), a.part_seg_rows) - s0) : 0;
        int most = sn;
        for (int off = 32; off > 0; off >>= 1) most = max(most, __shfl_xor(most, off));
        for (int q = 0; q < most; ++q) {
          float2 t[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            fft_in_index<N>(lane, i, b, n);
            t[i] = q < sn ? a.in_c[(int64_t)(s0 + q) * N + n] : make_float2(0.f, 0.f);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = cadd(v[i], t[i]);
        }
      } else {
        int p = 0;
        for (; p + 4 <= a.nparts; p += 4) {
          float2 t[4][16];
#pragma unroll
          for (int k = 0; k < 4; ++k) load_part(p + k, t[k]);
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = cadd(v[i], t[k][i]);
        }
        for (; p < a.nparts; ++p) {
          float2 t[16];
          load_part(p, t);
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = cadd(v[i], t[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        fft_in_index<N>(lane, i, b, n);
        const int64_t r = r0 + b;
        if (a.norm_cnt && r < a.nrows) {
          const int32_t c = a.norm_cnt[r * N + n];
          v[i] = c > 0 ? make_float2(v[i].x / (float)c, v[i].y / (float)c) : make_float2(0.f, 0.f);
        }
        if (a.sum_out && r < a.nrows) a.sum_out[r * N + n] = v[i];
        if (INV) v[i] = cconj(v[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        fft_in_index<N>(lane, i, b, n);
        const int64_t r = r0 + b;
        float2 x = make_float2(0.f, 0.f);
        if (r < a.nrows) {
          const int64_t e = r * N + n;
          if (in_mode == IN_C64) {
            x = a.in_c[e];
          } else if (in_mode == IN_HALF_C64) {
            // Hermitian row from its first N/2 + 1 entries: x(N - m) = conj x(m)
            const float2* hr = a.in_c + r * (N / 2 + 1);
            x = 2 * n <= N ? hr[n] : cconj(hr[N - n]);
          } else if (in_mode == IN_F32_PAIR) {
            x.x = a.in_f0[e] * a.s0;
            x.y = a.in_f1 ? a.in_f1[e] * a.s1 : 0.f;
          } else {
            x.x = (float)(a.in_d0[e] * (double)a.s0);
            x.y = a.in_d1 ? (float)(a.in_d1[e] * (double)a.s1) : 0.f;
          }
        }
        v[i] = INV ? cconj(x) : x;
      }
    }
    wave_fft<N>(v, buf, s_tw, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = cmul(INV ? cconj(v[i]) : v[i], a.osc);
    if (!transposed) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, m;
        fft_out_index<N>(lane, i, b, m);
        const int64_t r = r0 + b;
        if (r < a.nrows) {
          const int64_t e = r * N + m;
          if (out_mode == OUT_ROW_C64) a.out_c[e] = v[i];
          else if (out_mode == OUT_ROW_RE) a.out_f[e] = v[i].x;
          else a.out_f[e] = v[i].y;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, m;
        fft_out_index<N>(lane, i, b, m);
        buf[fft_pad(b * N + m)] = v[i];
      }
      __syncthreads();
      for (int u = threadIdx.x; u < TR * N; u += kRowThreads) {
        const int m = u / TR, rl = u % TR;
        const int w = rl / B, b = rl % B;
        const int64_t r = tile * TR + rl;
        if (r < a.nrows) {
          const float2 x = s_buf[w * kWaveStride + fft_pad(b * N + m)];
          const int64_t e = (int64_t)m * a.out_stride + r;
          if (out_mode == OUT_T_C64) a.out_c[e] = x;
          else if (out_mode == OUT_T_RE) a.out_f[e] = x.x;
          else a.out_f[e] = x.y;
        }
      }
      __syncthreads();
    }
  }
}

template <int N, int W>
static void launch_nw(bool inv, const RowFftArgs& a, int in, int out, hipStream_t s) {
  const int64_t tr = W * (1024 / N);
  const int64_t tiles = (a.nrows + tr - 1) / tr;
  const dim3 grid((unsigned)(tiles < 2048 ? tiles : 2048));
  if (in == IN_C64_SUM && a.part_seg) {
    if (inv)
      hipLaunchKernelGGL((k_row_fft<N, true, W, true, true>), grid, dim3(64 * W), 0, s, a, in, out);
    else
      hipLaunchKernelGGL((k_row_fft<N, false, W, true, true>), grid, dim3(64 * W), 0, s, a, in, out);
  } else if (in == IN_C64_SUM) {
    if (inv)
      hipLaunchKernelGGL((k_row_fft<N, true, W, true>), grid, dim3(64 * W), 0, s, a, in, out);
    else
      hipLaunchKernelGGL((k_row_fft<N, false, W, true>), grid, dim3(64 * W), 0, s, a, in, out);
  } else if (inv) {
    hipLaunchKernelGGL((k_row_fft<N, true, W, false>), grid, dim3(64 * W), 0, s, a, in, out);
  } else {
    hipLaunchKernelGGL((k_row_fft<N, false, W, false>), grid, dim3(64 * W), 0, s, a, in, out);
  }
}

template <int N>
static void launch_n(bool inv, const RowFftArgs& a, int in, int out, hipStream_t s) {
  // fewer than two 8-wave tiles per CU: 4-wave workgroups spread the rows over more CUs
  if (a.nrows < 2 * 256 * 8 * (1024 / N))
    launch_nw<N, 4>(inv, a, in, out, s);
  else
    launch_nw<N, 8>(inv, a, in, out, s);
}

// ---------------------------------------------------------------------------------------------
// Batched row FFTs of the lengths the wavefront FFT does not take (fft_generic.h): a workgroup
// loads RB rows into LDS (the input modes of k_row_fft, and real rows of counts), transforms them
// and writes them (the output modes of k_row_fft, and the row-transformed cube's transposed
// layout), grid-stride over batches of rows, its twiddle table filled once.  Transposed outputs
// are written rows-fastest (runs of RB consecutive rows per frequency).

bool scan_length_ok(int n) {
  if (fast_length(n)) return true;
  GPlan p;
  return n >= 16 && n % 2 == 0 && gen_plan(n, p);
}

__global__ void __launch_bounds__(kGenThreads) k_grow_fft(RowFftArgs a, GPlan p, int inv, int in_mode, int out_mode) {
  extern __shared__ float2 s_g[];  // twiddles [n], then rb rows of n
  const int n = p.n, rb = gen_rows_per_block(n);
  float2* tw = s_g;
  float2* buf = s_g + n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (in_mode == IN_C64_SUM && a.stats && blockIdx.x == 0) {
    // the fused sums' per-wave counters: pair count below bit 40, 8-byte loads above
    __shared__ unsigned long long s_red[2][kGenThreads / 64];
    unsigned long long c = 0, l = 0;
    for (int64_t i = threadIdx.x; i < a.nwcnt; i += blockDim.x) {
      c += a.wcnt[i] & ((1ull << 40) - 1);
      l += a.wcnt[i] >> 40;
    }
    for (int off = 32; off > 0; off >>= 1) {
      c += __shfl_xor(c, off);
      l += __shfl_xor(l, off);
    }
    if (lane == 0) {
      s_red[0][wave] = c;
      s_red[1][wave] = l;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      unsigned long long t = 0, u = 0;
      for (int w = 0; w < kGenThreads / 64; ++w) {
        t += s_red[0][w];
        u += s_red[1][w];
      }
      a.stats[threadIdx.x] = threadIdx.x == 0   ? t
                             : threadIdx.x == 1 ? (a.part_seg ? (unsigned long long)a.part_seg[a.nrows]
                                                              : (unsigned long long)a.stats_groups)
                             : threadIdx.x == 2 ? 8ull * u
                                                : (unsigned long long)a.stats_chunks;
    }
    if (threadIdx.x == 4 && a.ready_out) *a.ready_out = a.ready_val;
  }
  gen_twiddles(tw, n);
  __syncthreads();
  const int64_t nbatch = (a.nrows + rb - 1) / rb;
  const bool transposed = out_mode == OUT_T_C64 || out_mode == OUT_T_RE || out_mode == OUT_T_IM || out_mode == OUT_X;
  const int nh = n / 2 + 1;
  for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
    const int64_t r0 = bt * rb;
    for (int e = threadIdx.x; e < rb * n; e += blockDim.x) {
      const int rl = e / n, i = e % n;
      const int64_t r = r0 + rl;
      float2 x = make_float2(0.f, 0.f);
      if (r < a.nrows) {
        const int64_t el = r * n + i;
        if (in_mode == IN_C64) {
          x = a.in_c[el];
        } else if (in_mode == IN_C64_SUM) {
          if (a.part_seg) {
            const int64_t q0 = min(max(a.part_seg[r], (int64_t)0), a.part_seg_rows);
            const int64_t q1 = min(max(a.part_seg[r + 1], q0), a.part_seg_rows);
            for (int64_t q = q0; q < q1; ++q) x = cadd(x, a.in_c[q * n + i]);
          } else {
            for (int q = 0; q < a.nparts; ++q) x = cadd(x, a.in_c[(int64_t)q * a.part_stride + el]);
          }
          if (a.norm_cnt) {
            const int32_t cnt = a.norm_cnt[el];
            x = cnt > 0 ? make_float2(x.x / (float)cnt, x.y / (float)cnt) : make_float2(0.f, 0.f);
          }
          if (a.sum_out) a.sum_out[el] = x;
        } else if (in_mode == IN_HALF_C64) {
          const float2* hr = a.in_c + r * nh;
          x = 2 * i <= n ? hr[i] : cconj(hr[n - i]);
        } else if (in_mode == IN_F32_PAIR) {
          x.x = a.in_f0[el] * a.s0;
          x.y = a.in_f1 ? a.in_f1[el] * a.s1 : 0.f;
        } else if (in_mode == IN_F64_PAIR) {
          x.x = (float)(a.in_d0[el] * (double)a.s0);
          x.y = a.in_d1 ? (float)(a.in_d1[el] * (double)a.s1) : 0.f;
        } else if (in_mode == IN_U8) {
          x.x = (float)((const uint8_t*)a.in_u)[el];
        } else {
          x.x = (float)((const uint16_t*)a.in_u)[el];
        }
      }
      buf[e] = inv ? cconj(x) : x;
    }
    __syncthreads();
    gen_fft(buf, tw, p, rb);
    for (int e = threadIdx.x; e < rb * n; e += blockDim.x) {
      // transposed outputs rows-fastest, the others along the row
      const int rl = transposed ? e % rb : e / n, m = transposed ? e / rb : e % n;
      const int64_t r = r0 + rl;
      if (r >= a.nrows) continue;
      const float2 y = buf[rl * n + m];
      const float2 v = cmul(inv ? cconj(y) : y, a.osc);
      if (out_mode == OUT_ROW_C64) a.out_c[r * n + m] = v;
      else if (out_mode == OUT_ROW_RE) a.out_f[r * n + m] = v.x;
      else if (out_mode == OUT_ROW_IM) a.out_f[r * n + m] = v.y;
      else if (out_mode == OUT_T_C64) a.out_c[(int64_t)m * a.out_stride + r] = v;
      else if (out_mode == OUT_T_RE) a.out_f[(int64_t)m * a.out_stride + r] = v.x;
      else if (out_mode == OUT_T_IM) a.out_f[(int64_t)m * a.out_stride + r] = v.y;
      else if (m < nh) {
        const int64_t kd = r / a.xrows, y_ = r % a.xrows;
        a.out_c[(kd * nh + m) * a.xrows + y_] = v;
      }
    }
    __syncthreads();
  }
}

static int launch_generic(int n, bool inverse, RowIn in, RowOut out, const RowFftArgs& a, hipStream_t stream) {
  GPlan p;
  if (!gen_plan(n, p)) return STEM_EINVAL;
  const int rb = gen_rows_per_block(n);
  const int64_t batches = (a.nrows + rb - 1) / rb;
  const size_t lds = (size_t)(n + rb * n) * sizeof(float2);
  const int res = resident_blocks((const void*)k_grow_fft, kGenThreads, lds);
  const int64_t cap = res > 0 ? res : 1024;
  hipLaunchKernelGGL(k_grow_fft, dim3((unsigned)(batches < cap ? batches : cap)), dim3(kGenThreads), lds, stream, a,
                     p, inverse ? 1 : 0, (int)in, (int)out);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

int launch_row_fft(int n, bool inverse, RowIn in, RowOut out, const RowFftArgs& a, hipStream_t stream) {
  if (a.nrows <= 0) return STEM_OK;
  STEM_TRACE(a.tag ? a.tag : "row_fft", stream);
  if (!fast_length(n) || in == IN_U8 || in == IN_U16 || out == OUT_X) return launch_generic(n, inverse, in, out, a, stream);
  switch (n) {
    case 32: launch_n<32>(inverse, a, in, out, stream); break;
    case 64: launch_n<64>(inverse, a, in, out, stream); break;
    case 128: launch_n<128>(inverse, a, in, out, stream); break;
    case 256: launch_n<256>(inverse, a, in, out, stream); break;
    case 512: launch_n<512>(inverse, a, in, out, stream); break;
    case 1024: launch_n<1024>(inverse, a, in, out, stream); break;
    default: return STEM_EINVAL;
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// DPC: per-frequency recurrence (Sec. V).  C = FFT2(gx + i gy) row-major [my][mx]; the two real
// spectra are Gx = (C(q) + conj C(-q))/2, Gy = (C(q) - conj C(-q))/(2i).  With D = 2 pi i q and
// d = lam1 + |2 pi q|^2 + lam2 |2 pi q|^4:  Phi <- Phi + mu conj(D).(G - D Phi)/d, L times, in
// double; q = 0 and the Nyquist row/column are held at zero.

// ---------------------------------------------------------------------------------------------
// DPC integration in three passes over the packed gradient z = gx + i gy (Sec. V):
//  k_dpc_rows  rows ry: FFT along rx, split into the half spectra Gx, Gy along x (z(m) and
//              conj z(-m)), written transposed [mx][ry] for mx in [0, Nx/2];
//  k_dpc_cols  rows mx: FFT of both along ry, the per-frequency gradient descent (no mirror
//              element needed: Gx and Gy are separate), inverse FFT along my, written
//              transposed [ry][mx] (half spectrum along x);
//  then k_row_fft (IN_HALF_C64) rows ry: inverse along mx of the Hermitian row, real part / F.

template <int N, int W>
__global__ void __launch_bounds__(64 * W) k_dpc_rows(const double* __restrict__ c64, const float* __restrict__ c32,
                                                   int64_t plane, int ny, float g, float2* __restrict__ Ax,
                                                   float2* __restrict__ Ay) {
  constexpr int kThreads = 64 * W;
  constexpr int B = 1024 / N, TR = W * B, NH = N / 2 + 1;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[W * kWaveStride];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  fill_twiddles(s_tw, threadIdx.x, kThreads);
  __syncthreads();
  float2* buf = s_buf + wave * kWaveStride;
  const int ntiles = (ny + TR - 1) / TR;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * TR + wave * B;
    float2 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, n;
      fft_in_index<N>(lane, i, b, n);
      const int r = r0 + b;
      float2 x = make_float2(0.f, 0.f);
      if (r < ny) {
        const int64_t e = (int64_t)r * N + n;
        x = c64 ? make_float2((float)(c64[e] * (double)g), (float)(c64[plane + e] * (double)g))
                : make_float2(c32[e] * g, c32[plane + e] * g);
      }
      v[i] = x;
    }
    wave_fft<N>(v, buf, s_tw, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      fft_out_index<N>(lane, i, b, m);
      buf[fft_pad(b * N + m)] = v[i];
    }
    __syncthreads();
    for (int u = threadIdx.x; u < TR * NH; u += kThreads) {
      const int m = u / TR, rl = u % TR;
      const int w = rl / B, b = rl % B;
      const int r = tile * TR + rl;
      if (r < ny) {
        const float2* wb = s_buf + w * kWaveStride;
        const float2 z = wb[fft_pad(b * N + m)];
        const float2 zc = cconj(wb[fft_pad(b * N + ((N - m) & (N - 1)))]);
        Ax[(int64_t)m * ny + r] = cscale(cadd(z, zc), 0.5f);
        Ay[(int64_t)m * ny + r] = cscale(cmul_mi(csub(z, zc)), 0.5f);
      }
    }
    __syncthreads();
  }
}

template <int N, int W>
__global__ void __launch_bounds__(64 * W) k_dpc_cols(const float2* __restrict__ Ax, const float2* __restrict__ Ay,
                                                   int nx, double step, double mu, double lam1, double lam2,
                                                   int n_iter, float2* __restrict__ Q) {
  constexpr int kThreads = 64 * W;
  constexpr int B = 1024 / N, TR = W * B;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[W * kWaveStride];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  fill_twiddles(s_tw, threadIdx.x, kThreads);
  __syncthreads();
  float2* buf = s_buf + wave * kWaveStride;
  const int nh = nx / 2 + 1;
  const int ntiles = (nh + TR - 1) / TR;
  const double two_pi = 6.283185307179586476925286766559;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * TR + wave * B;  // rows are frequencies mx
    float2 vx[16], vy[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, n;
      fft_in_index<N>(lane, i, b, n);
      const int r = r0 + b;
      vx[i] = r < nh ? Ax[(int64_t)r * N + n] : make_float2(0.f, 0.f);
      vy[i] = r < nh ? Ay[(int64_t)r * N + n] : make_float2(0.f, 0.f);
    }
    wave_fft<N>(vx, buf, s_tw, lane);
    wave_fft<N>(vy, buf, s_tw, lane);
    // gradient descent per frequency (my, mx); the result goes to LDS in natural order
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, my;
      fft_out_index<N>(lane, i, b, my);
      const int mx = r0 + b;
      const int sy = my < (N + 1) / 2 ? my : my - N;
      const int sx = mx < (nx + 1) / 2 ? mx : mx - nx;
      const double qy = two_pi * ((double)sy / ((double)N * step));
      const double qx = two_pi * ((double)sx / ((double)nx * step));
      const double q2 = qx * qx + qy * qy;
      const double d = lam1 + q2 + lam2 * q2 * q2;
      const bool live = d != 0.0 && !(my == 0 && mx == 0) && my != N / 2 && mx != nx / 2 && mx < nh;
      double pr = 0.0, pi = 0.0;
      if (live) {
        const double gxr = vx[i].x, gxi = vx[i].y, gyr = vy[i].x, gyi = vy[i].y;
        const double md = mu / d;
        for (int l = 0; l < n_iter; ++l) {
          // residuals G - D Phi with D = i q, then conj(D) r = -i q r
          const double rxr = gxr + qx * pi, rxi = gxi - qx * pr;
          const double ryr = gyr + qy * pi, ryi = gyi - qy * pr;
          const double ur = qx * rxi + qy * ryi, ui = -(qx * rxr + qy * ryr);
          pr += md * ur;
          pi += md * ui;
        }
      }
      buf[fft_pad(b * N + my)] = make_float2((float)pr, (float)pi);
    }
    wave_lds_sync();
    // inverse along my: conj, forward transform, conj
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, n;
      fft_in_index<N>(lane, i, b, n);
      vx[i] = cconj(buf[fft_pad(b * N + n)]);
    }
    wave_lds_sync();
    wave_fft<N>(vx, buf, s_tw, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      fft_out_index<N>(lane, i, b, m);
      buf[fft_pad(b * N + m)] = cconj(vx[i]);
    }
    __syncthreads();
    // transposed write: Q[ry][mx], runs of TR frequencies mx
    for (int u = threadIdx.x; u < TR * N; u += kThreads) {
      const int m = u / TR, rl = u % TR;
      const int w = rl / B, b = rl % B;
      const int r = tile * TR + rl;
      if (r < nh) Q[(int64_t)m * nh + r] = s_buf[w * kWaveStride + fft_pad(b * N + m)];
    }
    __syncthreads();
  }
}

template <int N>
static void launch_dpc_rows(const double* c64, const float* c32, int64_t plane, int ny, float g, float2* Ax,
                            float2* Ay, hipStream_t s) {
  constexpr int W = 4;
  const int tiles = (ny + W * (1024 / N) - 1) / (W * (1024 / N));
  hipLaunchKernelGGL((k_dpc_rows<N, W>), dim3((unsigned)tiles), dim3(64 * W), 0, s, c64, c32, plane, ny, g, Ax, Ay);
}

template <int N>
static void launch_dpc_cols(const float2* Ax, const float2* Ay, int nx, double step, const stem_dpc& p, float2* Q,
                            hipStream_t s) {
  constexpr int W = 4;
  const int nh = nx / 2 + 1;
  const int tiles = (nh + W * (1024 / N) - 1) / (W * (1024 / N));
  hipLaunchKernelGGL((k_dpc_cols<N, W>), dim3((unsigned)tiles), dim3(64 * W), 0, s, Ax, Ay, nx, step, p.mu, p.lam1,
                     p.lam2, p.n_iter, Q);
}

// the three DPC passes for power-of-two lengths in [32, 1024]
static int launch_dpc(const double* c64, const float* c32, int64_t F, int ny, int nx, float g, double step,
                      const stem_dpc& p, float2* Ax, float2* Ay, float2* Q, float* phase, hipStream_t s) {
  {
    STEM_TRACE("dpc_rows", s);
    switch (nx) {
      case 32: launch_dpc_rows<32>(c64, c32, F, ny, g, Ax, Ay, s); break;
      case 64: launch_dpc_rows<64>(c64, c32, F, ny, g, Ax, Ay, s); break;
      case 128: launch_dpc_rows<128>(c64, c32, F, ny, g, Ax, Ay, s); break;
      case 256: launch_dpc_rows<256>(c64, c32, F, ny, g, Ax, Ay, s); break;
      case 512: launch_dpc_rows<512>(c64, c32, F, ny, g, Ax, Ay, s); break;
      case 1024: launch_dpc_rows<1024>(c64, c32, F, ny, g, Ax, Ay, s); break;
      default: return STEM_EINVAL;
    }
    STEM_LAUNCH_CHECK();
  }
  {
    STEM_TRACE("dpc_cols", s);
    switch (ny) {
      case 32: launch_dpc_cols<32>(Ax, Ay, nx, step, p, Q, s); break;
      case 64: launch_dpc_cols<64>(Ax, Ay, nx, step, p, Q, s); break;
      case 128: launch_dpc_cols<128>(Ax, Ay, nx, step, p, Q, s); break;
      case 256: launch_dpc_cols<256>(Ax, Ay, nx, step, p, Q, s); break;
      case 512: launch_dpc_cols<512>(Ax, Ay, nx, step, p, Q, s); break;
      case 1024: launch_dpc_cols<1024>(Ax, Ay, nx, step, p, Q, s); break;
      default: return STEM_EINVAL;
    }
    STEM_LAUNCH_CHECK();
  }
  // inverse along mx of the Hermitian rows, real part / F -> phase[ry][rx]
  RowFftArgs a{};
  a.nrows = ny;
  a.in_c = Q;
  a.out_f = phase;
  a.osc = make_float2((float)(1.0 / (double)F), 0.f);
  a.tag = "dpc_fft";
  return launch_row_fft(nx, true, IN_HALF_C64, OUT_ROW_RE, a, s);
}

// ---------------------------------------------------------------------------------------------
// DPC for the other scan lengths, in five passes of the generic FFT and one per-frequency pass:
// rows ry of z = g (COM_x + i COM_y) transformed along rx and written transposed [mx][ry]; rows mx
// transformed along ry in place (C = FFT2 z, column-major [mx][my]); the descent per frequency from
// Gx = (C(q) + conj C(-q))/2 and Gy = (C(q) - conj C(-q))/(2i) into Phi; the inverse along my,
// written transposed [ry][mx]; the inverse along mx, real part / F.

__global__ void __launch_bounds__(256) k_dpc_descent(const float2* __restrict__ C, int ny, int nx, double step,
                                                     double mu, double lam1, double lam2, int n_iter,
                                                     float2* __restrict__ Phi) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)ny * nx) return;
  const int mx = (int)(q / ny), my = (int)(q % ny);
  const float2 c = C[q];
  const float2 cm = cconj(C[(int64_t)((nx - mx) % nx) * ny + (ny - my) % ny]);
  const double two_pi = 6.283185307179586476925286766559;
  const int sy = my < (ny + 1) / 2 ? my : my - ny;
  const int sx = mx < (nx + 1) / 2 ? mx : mx - nx;
  const double qy = two_pi * ((double)sy / ((double)ny * step));
  const double qx = two_pi * ((double)sx / ((double)nx * step));
  const double q2 = qx * qx + qy * qy;
  const double d = lam1 + q2 + lam2 * q2 * q2;
  const bool live = d != 0.0 && !(my == 0 && mx == 0) && 2 * my != ny && 2 * mx != nx;
  double pr = 0.0, pi = 0.0;
  if (live) {
    // Gx = (c + cm)/2, Gy = (c - cm)/(2i)
    const float2 gx = make_float2(0.5f * (c.x + cm.x), 0.5f * (c.y + cm.y));
    const float2 gy = make_float2(0.5f * (c.y - cm.y), -0.5f * (c.x - cm.x));
    const double gxr = gx.x, gxi = gx.y, gyr = gy.x, gyi = gy.y;
    const double md = mu / d;
    for (int l = 0; l < n_iter; ++l) {
      // residuals G - D Phi with D = i q, then conj(D) r = -i q r
      const double rxr = gxr + qx * pi, rxi = gxi - qx * pr;
      const double ryr = gyr + qy * pi, ryi = gyi - qy * pr;
      const double ur = qx * rxi + qy * ryi, ui = -(qx * rxr + qy * ryr);
      pr += md * ur;
      pi += md * ui;
    }
  }
  Phi[q] = make_float2((float)pr, (float)pi);
}

static int launch_dpc_generic(const double* c64, const float* c32, int64_t F, int ny, int nx, float g, double step,
                              const stem_dpc& p, float2* A, float2* B, float* phase, hipStream_t s) {
  RowFftArgs a{};
  a.nrows = ny;
  if (c64) {
    a.in_d0 = c64;
    a.in_d1 = c64 + F;
  } else {
    a.in_f0 = c32;
    a.in_f1 = c32 + F;
  }
  a.s0 = a.s1 = g;
  a.out_c = A;
  a.out_stride = ny;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "dpc_fft";
  int st = launch_row_fft(nx, false, c64 ? IN_F64_PAIR : IN_F32_PAIR, OUT_T_C64, a, s);
  if (st) return st;
  a = RowFftArgs{};
  a.nrows = nx;
  a.in_c = A;
  a.out_c = A;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "dpc_fft";
  if ((st = launch_row_fft(ny, false, IN_C64, OUT_ROW_C64, a, s))) return st;
  {
    STEM_TRACE("dpc_descent", s);
    hipLaunchKernelGGL(k_dpc_descent, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, s, A, ny, nx, step, p.mu,
                       p.lam1, p.lam2, p.n_iter, B);
    STEM_LAUNCH_CHECK();
  }
  a = RowFftArgs{};
  a.nrows = nx;
  a.in_c = B;
  a.out_c = A;
  a.out_stride = nx;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "dpc_fft";
  if ((st = launch_row_fft(ny, true, IN_C64, OUT_T_C64, a, s))) return st;
  a = RowFftArgs{};
  a.nrows = ny;
  a.in_c = A;
  a.out_f = phase;
  a.osc = make_float2((float)(1.0 / (double)F), 0.f);
  a.tag = "dpc_fft";
  return launch_row_fft(nx, true, IN_C64, OUT_ROW_RE, a, s);
}

}  // namespace stem

// ---------------------------------------------------------------------------------------------
// C ABI

using namespace stem;

extern "C" size_t com_dpc_workspace_bytes(const stem_scan* scan) {
  if (!scan || scan->ny <= 0 || scan->nx <= 0) return 0;
  if (fast_length(scan->ny) && fast_length(scan->nx))
    // the half spectra Gx, Gy along x and the half-spectrum result, (Nx/2+1) Ny complex64 each
    return 3 * align256((size_t)scan->ny * (scan->nx / 2 + 1) * sizeof(float2));
  // the other lengths: the full transform of z and the descent's result, F complex64 each
  return 2 * align256((size_t)scan->ny * scan->nx * sizeof(float2));
}

static int run_com_dpc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                       const stem_det* det, const stem_scan* scan, const stem_optics* optics, const stem_dpc* dpc,
                       double* d_com64, float* d_com32, int32_t* d_counts, float* d_phase, void* ws,
                       size_t ws_bytes, int32_t* d_status, void* stream_) {
  if (!d_idx || !d_off || !det || !scan) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  if (scan->ny <= 0 || scan->nx <= 0) return STEM_EINVAL;
  const int64_t F = (int64_t)scan->ny * scan->nx;
  if (frame0 < 0 || n_frames < 0 || frame0 + n_frames > F) return STEM_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (d_phase) {
    if (!optics || !dpc || (!d_com64 && !d_com32)) return STEM_EINVAL;
    if (!scan_length_ok(scan->ny) || !scan_length_ok(scan->nx)) return STEM_EINVAL;
    if (!(scan->step > 0) || !(optics->dk > 0) || dpc->n_iter < 0) return STEM_EINVAL;
    if (!ws || ws_bytes < com_dpc_workspace_bytes(scan) || ((uintptr_t)ws & 255)) return STEM_EWORKSPACE;
  }
  int st = launch_com(d_idx, d_off, frame0, n_frames, *det, F, d_com64, d_com32, d_counts, d_status, stream);
  if (st != STEM_OK || !d_phase) return st;

  const int ny = scan->ny, nx = scan->nx;
  const float g = (float)(2.0 * 3.14159265358979323846 * optics->dk);
  if (!fast_length(ny) || !fast_length(nx)) {
    float2* A = (float2*)ws;
    float2* B = (float2*)((char*)ws + align256((size_t)F * sizeof(float2)));
    return launch_dpc_generic(d_com64, d_com64 ? nullptr : d_com32, F, ny, nx, g, scan->step, *dpc, A, B, d_phase,
                              stream);
  }
  const size_t half = align256((size_t)ny * (nx / 2 + 1) * sizeof(float2));
  float2* Ax = (float2*)ws;
  float2* Ay = (float2*)((char*)ws + half);
  float2* Q = (float2*)((char*)ws + 2 * half);
  return launch_dpc(d_com64, d_com64 ? nullptr : d_com32, F, ny, nx, g, scan->step, *dpc, Ax, Ay, Q, d_phase, stream);
}

extern "C" int com_dpc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                       const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                       const stem_dpc* dpc, double* d_com64, float* d_com32, int32_t* d_counts,
                       float* d_phase, void* ws, size_t ws_bytes, int32_t* d_status, void* stream_) {
  return run_com_dpc(d_idx, d_off, frame0, n_frames, det, scan, optics, dpc, d_com64, d_com32, d_counts, d_phase, ws,
                     ws_bytes, d_status, stream_);
}

// ---------------------------------------------------------------------------------------------
// com_dpc without a caller workspace: the DPC integration's half-spectrum planes live in a
// file-scope device array (one copy per GPU, held until the process ends).  In host code the
// array's name is not a device address: its address on each device is looked up once, with that
// device current, and only that pointer is passed to kernels.

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch`, looked up on its first use (nullptr if the lookup fails)
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t com_dpc_noalloc_max_workspace(void) { return kNoAllocScratchBytes; }

extern "C" int com_dpc_noalloc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                               const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                               const stem_dpc* dpc, double* d_com64, float* d_com32, int32_t* d_counts,
                               float* d_phase, int32_t* d_status, void* stream_) {
  void* ws = nullptr;
  if (d_phase) {
    if (!scan) return STEM_EINVAL;
    if (com_dpc_workspace_bytes(scan) > kNoAllocScratchBytes) return STEM_EWORKSPACE;
    ws = scratch_on_current_device();
    if (!ws) return STEM_EHIP;
  }
  return run_com_dpc(d_idx, d_off, frame0, n_frames, det, scan, optics, dpc, d_com64, d_com32, d_counts, d_phase, ws,
                     d_phase ? kNoAllocScratchBytes : 0, d_status, stream_);
}
