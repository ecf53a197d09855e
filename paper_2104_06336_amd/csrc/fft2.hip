// Batched row FFTs (power-of-two lengths 32..1024) and the centre-of-mass DPC path
// (Eq. 4 and the regularised Fourier gradient descent of Sec. V).
//
// k_row_fft: a workgroup of W = 8 waves (4 when there are too few rows to give every CU a
// workgroup); each wave transforms B = 1024/N rows at a time with the wavefront FFT of
// fft_wave.h.  Row-major outputs are stored straight from registers; transposed outputs
// (element (r, m) -> out[m*stride + r]) are first staged in the waves' LDS buffers so that the
// workgroup writes runs of W B consecutive rows per frequency.
#include "common.h"
#include "fft_wave.h"
#include "kernels.h"
#include "trace.h"

namespace stem {

constexpr int kWaveStride = kFftLds + 4;  // float2 per wave buffer; the +4 staggers LDS banks

// SUM: the input is the sum of a.nparts partial planes (in_mode IN_C64_SUM), read four at a time;
// a separate instantiation, so that the other input modes keep their lower register count.
template <int N, bool INV, int W, bool SUM>
__global__ void __launch_bounds__(64 * W) k_row_fft(RowFftArgs a, int in_mode, int out_mode) {
  constexpr int kRowThreads = 64 * W;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[W * kWaveStride];
  constexpr int B = 1024 / N;
  constexpr int TR = W * B;  // rows per tile
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        fft_in_index<N>(lane, i, b, n);
        const int64_t r = r0 + b;
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
  if (in == IN_C64_SUM) {
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

int launch_row_fft(int n, bool inverse, RowIn in, RowOut out, const RowFftArgs& a, hipStream_t stream) {
  if (a.nrows <= 0) return STEM_OK;
  STEM_TRACE(a.tag ? a.tag : "row_fft", stream);
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

__global__ void __launch_bounds__(256) k_dpc_update(const float2* __restrict__ C, float2* __restrict__ Phi,
                                                    int ny, int nx, double step, double mu, double lam1,
                                                    double lam2, int n_iter) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ny * nx) return;
  const int my = (int)(e / nx), mx = (int)(e % nx);
  const int myn = (ny - my) % ny, mxn = (nx - mx) % nx;
  const float2 c = C[e], cm = C[(int64_t)myn * nx + mxn];
  // Gx = (c + conj cm)/2, Gy = (c - conj cm)/(2i)
  const double gxr = 0.5 * ((double)c.x + cm.x), gxi = 0.5 * ((double)c.y - cm.y);
  const double dyr = 0.5 * ((double)c.x - cm.x), dyi = 0.5 * ((double)c.y + cm.y);
  const double gyr = dyi, gyi = -dyr;  // (a + ib)/i = b - ia
  const int sy = my < (ny + 1) / 2 ? my : my - ny;
  const int sx = mx < (nx + 1) / 2 ? mx : mx - nx;
  const double two_pi = 6.283185307179586476925286766559;
  const double qy = two_pi * ((double)sy / ((double)ny * step));
  const double qx = two_pi * ((double)sx / ((double)nx * step));
  const double q2 = qx * qx + qy * qy;
  const double d = lam1 + q2 + lam2 * q2 * q2;
  const bool live = d != 0.0 && !(my == 0 && mx == 0) && !((ny % 2 == 0) && my == ny / 2) &&
                    !((nx % 2 == 0) && mx == nx / 2);
  double pr = 0.0, pi = 0.0;
  if (live) {
    const double md = mu / d;  // the step size over the regularised denominator, fixed per frequency
    for (int l = 0; l < n_iter; ++l) {
      // residuals G - D Phi with D = i q:  i q (pr + i pi) = -q pi + i q pr
      const double rxr = gxr + qx * pi, rxi = gxi - qx * pr;
      const double ryr = gyr + qy * pi, ryi = gyi - qy * pr;
      // conj(D) r = -i q r = q ri - i q rr
      const double ur = qx * rxi + qy * ryi, ui = -(qx * rxr + qy * ryr);
      pr += md * ur;
      pi += md * ui;
    }
  }
  Phi[e] = make_float2((float)pr, (float)pi);
}

int launch_dpc_update(const float2* C, float2* Phi, int ny, int nx, double step, const stem_dpc& p,
                      hipStream_t stream) {
  const int64_t n = (int64_t)ny * nx;
  STEM_TRACE("dpc_update", stream);
  hipLaunchKernelGGL(k_dpc_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, C, Phi, ny, nx,
                     step, p.mu, p.lam1, p.lam2, p.n_iter);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem

// ---------------------------------------------------------------------------------------------
// C ABI

using namespace stem;

extern "C" size_t com_dpc_workspace_bytes(const stem_scan* scan) {
  if (!scan || scan->ny <= 0 || scan->nx <= 0) return 0;
  return 2 * align256((size_t)scan->ny * scan->nx * sizeof(float2));
}

extern "C" int com_dpc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                       const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                       const stem_dpc* dpc, double* d_com64, float* d_com32, int32_t* d_counts,
                       float* d_phase, void* ws, size_t ws_bytes, int32_t* d_status, void* stream_) {
  if (!d_idx || !d_off || !det || !scan) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  if (scan->ny <= 0 || scan->nx <= 0) return STEM_EINVAL;
  const int64_t F = (int64_t)scan->ny * scan->nx;
  if (frame0 < 0 || n_frames < 0 || frame0 + n_frames > F) return STEM_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (d_phase) {
    if (!optics || !dpc || (!d_com64 && !d_com32)) return STEM_EINVAL;
    if (!is_pow2_in(scan->ny, 32, 1024) || !is_pow2_in(scan->nx, 32, 1024)) return STEM_EINVAL;
    if (!(scan->step > 0) || !(optics->dk > 0) || dpc->n_iter < 0) return STEM_EINVAL;
    if (!ws || ws_bytes < com_dpc_workspace_bytes(scan) || ((uintptr_t)ws & 255)) return STEM_EWORKSPACE;
  }
  int st = launch_com(d_idx, d_off, frame0, n_frames, *det, F, d_com64, d_com32, d_counts, d_status, stream);
  if (st != STEM_OK || !d_phase) return st;

  const int ny = scan->ny, nx = scan->nx;
  float2* A = (float2*)ws;
  float2* Bb = (float2*)((char*)ws + align256((size_t)F * sizeof(float2)));
  const float g = (float)(2.0 * 3.14159265358979323846 * optics->dk);
  RowFftArgs a{};
  // pass 1: rows (ry) of gx + i gy along rx -> A[mx][ry]
  a.nrows = ny;
  if (d_com64) {
    a.in_d0 = d_com64;
    a.in_d1 = d_com64 + F;
  } else {
    a.in_f0 = d_com32;
    a.in_f1 = d_com32 + F;
  }
  a.s0 = a.s1 = g;
  a.out_c = A;
  a.out_stride = ny;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "dpc_fft";
  st = launch_row_fft(nx, false, d_com64 ? IN_F64_PAIR : IN_F32_PAIR, OUT_T_C64, a, stream);
  if (st) return st;
  // pass 2: rows (mx) of A along ry -> Bb[my][mx]
  a = RowFftArgs{};
  a.nrows = nx;
  a.in_c = A;
  a.out_c = Bb;
  a.out_stride = nx;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "dpc_fft";
  if ((st = launch_row_fft(ny, false, IN_C64, OUT_T_C64, a, stream))) return st;
  // gradient descent per frequency: Bb -> A (Phi, [my][mx])
  if ((st = launch_dpc_update(Bb, A, ny, nx, scan->step, *dpc, stream))) return st;
  // pass 3: inverse along mx -> Bb[rx][my]
  a.nrows = ny;
  a.in_c = A;
  a.out_c = Bb;
  a.out_stride = ny;
  if ((st = launch_row_fft(nx, true, IN_C64, OUT_T_C64, a, stream))) return st;
  // pass 4: inverse along my -> phase[ry][rx] = Re / N_R
  a = RowFftArgs{};
  a.nrows = nx;
  a.in_c = Bb;
  a.out_f = d_phase;
  a.out_stride = nx;
  a.osc = make_float2((float)(1.0 / (double)F), 0.f);
  a.tag = "dpc_fft";
  return launch_row_fft(ny, true, IN_C64, OUT_T_RE, a, stream);
}
