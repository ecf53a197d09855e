// Eq. 3 and its adjoint from the stored double-overlap values of G (the pruned array whose layout
// ssb_fused.h describes): the refocus sum of Sec. IV (only the summation runs again) and the
// adjoint without any transform.
//
// A wave owns one scan-frequency column mx of the whole plane (Qx = ix(mx) sx, mx in [0, Nx)) and
// a group of pixels.  The lanes first gather the descriptors of 64 pixels at a time (start and
// length of the pixel's run for this column, the set's first row frequency and hole, Kc and
// chi(Kc) + theta) into LDS; the wave then streams each pixel's run of stored values, 64 lanes x 4
// entries per round (contiguous, coalesced loads), and adds every value, times its phase factor,
// into the column's T kept in LDS (one slot per row frequency my: the entries of a run have
// distinct my, so no two lanes touch one slot).  The partial T of the group goes to part[g]
// (column-major [mx][my], summed by the phase pass like the fused sum's).
//
// FULLG: the runs are read from a block of full half-spectrum columns of G instead (pixel kd's
// column c at X + ((kd - xk0) (Nx/2+1) + c) Ny; a column mx > Nx/2 is the conjugate of column
// Nx - mx at -my): the sums of the scan lengths the fused kernels do not take, whose G comes from
// separate row and column transforms.  With PWRITE the values read are also stored as the pruned
// array.
#pragma once

#include "ssb_fused.h"

namespace stem {

struct RunDesc {
  int64_t e0;     // first entry of the run
  int32_t len;    // entries (0: the pixel has no pair in this column)
  int32_t a0;     // signed row frequency of the first entry
  int32_t split;  // entries before the hole of the set
  int32_t hl;     // hole length (0: none)
  double kx, ky, kch;
};

// LDS bytes of one wave of the pruned kernels: the column of T (of Tbar for the adjoint), the 64
// descriptors and the adjoint's 64 dL/dtheta partials
__host__ __device__ inline size_t pruned_wave_lds(int ny, bool adjoint) {
  return (size_t)ny * sizeof(float2) + 64 * sizeof(RunDesc) + (adjoint ? 64 * sizeof(float) : 0);
}

// descriptors of pixels [kb, kb + 64) for column mx (lane j takes pixel kb + j); fullg: run lengths
// from the sets (e0 = the pruned array's offset when it exists)
__device__ __forceinline__ void gather_runs(const YArgs& a, const Optics& o, int kb, int kd_b, int mx, int lane,
                                            bool general, bool fullg, RunDesc* rd) {
  const int nx = a.nx, nc = nx / 2 + 1;
  const bool mir = 2 * mx > nx;
  const int c = mir ? nx - mx : mx;
  const int kd = kb + lane;
  RunDesc d{0, 0, 0, 0, 0, 0.0, 0.0, 0.0};
  if (kd < kd_b) {
    ColSet sd, sm;
    load_colsets(a.cst, (int64_t)kd * nc + c, sd, sm);
    const ColSet s = mir ? sm : sd;
    const int h0 = max(s.a0, s.b0), h1 = min(s.a1, s.b1);
    if (fullg) {
      d.e0 = a.poff ? a.poff[(int64_t)kd * nx + mx] : 0;
      d.len = set_size(s);
    } else {
      const int64_t e0 = a.poff[(int64_t)kd * nx + mx], e1 = a.poff[(int64_t)kd * nx + mx + 1];
      // entries are read only inside the array (a state whose FINALIZE never ran reads nothing
      // out of bounds)
      const bool ok = e0 >= 0 && e1 >= e0 && e1 <= a.pcap;
      d.e0 = ok ? e0 : 0;
      d.len = ok ? (int)(e1 - e0) : 0;
    }
    d.a0 = s.a0;
    d.hl = h0 <= h1 ? h1 - h0 + 1 : 0;
    d.split = h0 - s.a0;
    if (general) {
      const double2 k = a.kc[kd];
      d.kx = k.x;
      d.ky = k.y;
      d.kch = a.kchi[kd];
    }
  }
  rd[lane] = d;
  (void)o;
}

// Signed row frequency of entry u of run r.
__device__ __forceinline__ int run_iy(const RunDesc& r, int u) { return r.a0 + u + ((r.hl && u >= r.split) ? r.hl : 0); }

// One round of a run: entries u0 + lane + 64 q (q < 4) of run r of pixel kd, column mx (0 past its
// end), from the pruned array or (FULLG) from the full columns of G.
template <bool FULLG>
__device__ __forceinline__ void load_round(const YArgs& a, const RunDesc& r, int kd, int mx, int ny, int u0, int lane,
                                           float2* gv) {
  const int nx = a.nx, nh = nx / 2 + 1;
  const bool mir = 2 * mx > nx;
  const float2* col =
      FULLG ? a.X + ((int64_t)(kd - a.xk0) * nh + (mir ? nx - mx : mx)) * ny : nullptr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = u0 + lane + 64 * q;
    float2 x = make_float2(0.f, 0.f);
    if (u < r.len) {
      if constexpr (FULLG) {
        const int iy = run_iy(r, u);
        const int my = iy < 0 ? iy + ny : iy;
        x = mir ? cconj(col[(ny - my) % ny]) : col[my];
      } else {
        x = a.pg[r.e0 + u];
      }
    }
    gv[q] = x;
  }
}

// The next run with entries after pixel slot j of the batch (nb if none).
__device__ __forceinline__ int next_run(const RunDesc* rd, int j, int nb) {
  for (++j; j < nb; ++j)
    if (rd[j].len > 0) return j;
  return nb;
}

// T of column mx over the pixels [kd_a, kd_b) of group g from the stored values.  CHI0: every phase
// factor is exactly 1.  The first rounds of the next two runs are loaded while a run is summed.
template <bool CHI0, bool FULLG, bool PWRITE>
__global__ void __launch_bounds__(256) k_psum(YArgs a, Optics o, int ny) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* wl_ = s_dyn + (size_t)wave * pruned_wave_lds(ny, false);
  float2* t = (float2*)wl_;
  RunDesc* rd = (RunDesc*)(wl_ + (size_t)ny * sizeof(float2));
  const int nx = a.nx;
  const int g = blockIdx.x % a.ngroups;
  const int mx = (blockIdx.x / a.ngroups) * W + wave;
  const int64_t wid = (int64_t)blockIdx.x * W + wave;
  if (mx >= nx) {
    if (lane == 0 && !a.accumulate) a.wcnt[wid] = 0ull;
    return;
  }
  for (int i = lane; i < ny; i += 64) t[i] = make_float2(0.f, 0.f);
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const int kd_a = a.k0 + (int)((int64_t)(a.k1 - a.k0) * g / a.ngroups);
  const int kd_b = a.k0 + (int)((int64_t)(a.k1 - a.k0) * (g + 1) / a.ngroups);
  unsigned long long cnt = 0;
  for (int kb = kd_a; kb < kd_b; kb += 64) {
    gather_runs(a, o, kb, kd_b, mx, lane, !CHI0, FULLG, rd);
    wave_lds_sync();
    const int nb = min(64, kd_b - kb);
    int j = next_run(rd, -1, nb);
    int j1 = j < nb ? next_run(rd, j, nb) : nb;
    float2 g0[4], g1[4];
    if (j < nb) load_round<FULLG>(a, rd[j], kb + j, mx, ny, 0, lane, g0);
    if (j1 < nb) load_round<FULLG>(a, rd[j1], kb + j1, mx, ny, 0, lane, g1);
    while (j < nb) {
      const RunDesc r = rd[j];
      const int j2 = j1 < nb ? next_run(rd, j1, nb) : nb;
      float2 g2[4];
      if (j2 < nb) load_round<FULLG>(a, rd[j2], kb + j2, mx, ny, 0, lane, g2);
      cnt += (unsigned long long)r.len;
      ChiCol ch{};
      if constexpr (!CHI0) ch = chi_column(o.lk * (r.kx - qx), o);
      for (int u0 = 0; u0 < r.len; u0 += 256) {
        float2 gv[4];
        if (u0 == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) gv[q] = g0[q];
        } else {
          load_round<FULLG>(a, r, kb + j, mx, ny, u0, lane, gv);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = u0 + lane + 64 * q;
          if (u >= r.len) continue;
          const int iy = run_iy(r, u);
          const int my = iy < 0 ? iy + ny : iy;
          float2 val = gv[q];
          if constexpr (PWRITE) {
            if (r.e0 + u < a.pcap) a.pgw[r.e0 + u] = val;
          }
          if constexpr (!CHI0) {
            const double wy = o.lk * (r.ky - (double)iy * o.sy);
            const float2 e = expi_reduced(chi_eval(ch, wy) - r.kch);
            val = make_float2(gv[q].x * e.x - gv[q].y * e.y, gv[q].x * e.y + gv[q].y * e.x);
          }
          t[my] = cadd(t[my], val);
        }
      }
      j = j1;
      j1 = j2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        g0[q] = g1[q];
        g1[q] = g2[q];
      }
    }
    wave_lds_sync();  // the descriptors are rewritten for the next 64 pixels
  }
  float2* pgp = a.part + (int64_t)g * nx * ny + (int64_t)mx * ny;
  for (int i = lane; i < ny; i += 64) pgp[i] = a.accumulate ? cadd(pgp[i], t[i]) : t[i];
  unsigned long long cc = cnt + (cnt << kLoadShift);  // one 8-byte load per pair
  if (lane == 0) a.wcnt[wid] = a.accumulate ? a.wcnt[wid] + cc : cc;
}

// FP64 sum over the 64 lanes of a wave (every lane active), returned to every lane
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Adjoint of Eq. 3 from the stored values: for every pair, z = G e^{i psi}, w = Re(conj(Tbar(Q)) i z);
// per (pixel, column) run the moments M_n = sum w wy^n (n = 0..4) give the eight dL/dc terms (the
// B_j(K - Q) are polynomials in wy along a column, see k_yadjoint); dL/dtheta[kd] = -sum w.
// Partials: pdc[wave][8] (FP64), pdth[mx][kd] (FP32; one writer per entry).
template <bool FULLG>
__global__ void __launch_bounds__(256) k_padj(YArgs a, Optics o, int ny) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* wl_ = s_dyn + (size_t)wave * pruned_wave_lds(ny, true);
  float2* tb = (float2*)wl_;
  RunDesc* rd = (RunDesc*)(wl_ + (size_t)ny * sizeof(float2));
  float* wth = (float*)(rd + 64);
  const int nx = a.nx;
  const int g = blockIdx.x % a.ngroups;
  const int mx = (blockIdx.x / a.ngroups) * W + wave;
  const int64_t wid = (int64_t)blockIdx.x * W + wave;
  if (mx >= nx) {
    if (lane < 8 && !a.accumulate) a.pdc[wid * 8 + lane] = 0.0;
    return;
  }
  for (int i = lane; i < ny; i += 64) tb[i] = a.Tbt[(int64_t)mx * ny + i];
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const double s2pi = 6.283185307179586476925286766559 / o.lam;
  const int kd_a = a.k0 + (int)((int64_t)(a.k1 - a.k0) * g / a.ngroups);
  const int kd_b = a.k0 + (int)((int64_t)(a.k1 - a.k0) * (g + 1) / a.ngroups);
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  float* pth = a.pdth + (int64_t)mx * a.n_k;
  for (int kb = kd_a; kb < kd_b; kb += 64) {
    gather_runs(a, o, kb, kd_b, mx, lane, true, FULLG, rd);
    wave_lds_sync();
    const int nb = min(64, kd_b - kb);
    if (lane < nb) wth[lane] = 0.f;  // pixels without pairs in this column
    int j = next_run(rd, -1, nb);
    int j1 = j < nb ? next_run(rd, j, nb) : nb;
    float2 g0[4], g1[4];
    if (j < nb) load_round<FULLG>(a, rd[j], kb + j, mx, ny, 0, lane, g0);
    if (j1 < nb) load_round<FULLG>(a, rd[j1], kb + j1, mx, ny, 0, lane, g1);
    while (j < nb) {
      const RunDesc r = rd[j];
      const int j2 = j1 < nb ? next_run(rd, j1, nb) : nb;
      float2 g2[4];
      if (j2 < nb) load_round<FULLG>(a, rd[j2], kb + j2, mx, ny, 0, lane, g2);
      const double wx = o.lk * (r.kx - qx);
      const ChiCol ch = chi_column(wx, o);
      double M0 = 0.0, M1 = 0.0, M2 = 0.0, M3 = 0.0, M4 = 0.0;
      for (int u0 = 0; u0 < r.len; u0 += 256) {
        float2 gv[4];
        if (u0 == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) gv[q] = g0[q];
        } else {
          load_round<FULLG>(a, r, kb + j, mx, ny, u0, lane, gv);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = u0 + lane + 64 * q;
          if (u >= r.len) continue;
          const int iy = run_iy(r, u);
          const int my = iy < 0 ? iy + ny : iy;
          const double wy = o.lk * (r.ky - (double)iy * o.sy);
          const float2 e = expi_reduced(chi_eval(ch, wy) - r.kch);
          const float2 z = make_float2(gv[q].x * e.x - gv[q].y * e.y, gv[q].x * e.y + gv[q].y * e.x);
          const float2 tq = tb[my];
          double t = (double)(tq.x * (-z.y) + tq.y * z.x);
          M0 += t;
          t *= wy;
          M1 += t;
          t *= wy;
          M2 += t;
          t *= wy;
          M3 += t;
          t *= wy;
          M4 += t;
        }
      }
      // this lane's sum over its pairs of w B_j(K - Q), B_j as polynomials in wy
      const double x2 = wx * wx, x3 = x2 * wx, x4 = x2 * x2;
      dc[0] += 0.5 * s2pi * (x2 * M0 + M2);
      dc[1] += 0.5 * s2pi * (x2 * M0 - M2);
      dc[2] += s2pi * (wx * M1);
      dc[3] += (s2pi / 3.0) * (x3 * M0 + wx * M2);
      dc[4] += (s2pi / 3.0) * (x2 * M1 + M3);
      dc[5] += (s2pi / 3.0) * (x3 * M0 - 3.0 * wx * M2);
      dc[6] += (s2pi / 3.0) * (3.0 * x2 * M1 - M3);
      dc[7] += 0.25 * s2pi * (x4 * M0 + 2.0 * x2 * M2 + M4);
      // sum over the run of w B_j(K): B_j(K) times the run's sum of w, on lane 0
      const double wsum = wave_sum_f64(M0);
      if (lane == 0) {
        double bk[8];
        chi_basis(r.kx, r.ky, o, bk);
#pragma unroll
        for (int q = 0; q < 8; ++q) dc[q] -= bk[q] * wsum;
        wth[j] = (float)-wsum;
      }
      j = j1;
      j1 = j2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        g0[q] = g1[q];
        g1[q] = g2[q];
      }
    }
    wave_lds_sync();
    if (lane < nb) pth[kb + lane] = wth[lane];
    wave_lds_sync();  // the descriptors and partials are rewritten for the next 64 pixels
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double t = wave_sum_f64(dc[j]);
    if (lane == 0) a.pdc[wid * 8 + j] = a.accumulate ? a.pdc[wid * 8 + j] + t : t;
  }
}

// waves per workgroup of the pruned kernels for a column of ny row frequencies (LDS <= 64 KB)
inline int pruned_waves(int ny, bool adjoint) {
  int w = 4;
  while (w > 1 && (size_t)w * pruned_wave_lds(ny, adjoint) > (64u << 10)) w >>= 1;
  return w;
}

inline dim3 pruned_grid(int nx, int ngroups, int w) { return dim3((unsigned)(((nx + w - 1) / w) * ngroups)); }

// waves a launch of the pruned kernels writes partials for (wave index blockIdx.x * w + wave)
inline int64_t pruned_launch_waves(int ny, int nx, int ngroups, bool adjoint) {
  const int w = pruned_waves(ny, adjoint);
  return (int64_t)((nx + w - 1) / w) * ngroups * w;
}

// fullg: the runs from full columns of G at a.X (pixels from a.xk0); pwrite: also store the values
// as the pruned array
inline int launch_psum(int ny, const YArgs& a, const Optics& o, int chi0, bool fullg, bool pwrite, hipStream_t s) {
  const int w = pruned_waves(ny, false);
  const size_t lds = (size_t)w * pruned_wave_lds(ny, false);
  const dim3 grid = pruned_grid(a.nx, a.ngroups, w), blk(64 * w);
  STEM_TRACE(fullg ? "ssb_gsum" : "ssb_reduce", s);
  auto go = [&](auto c0, auto fg, auto pw) {
    hipLaunchKernelGGL((k_psum<decltype(c0)::value, decltype(fg)::value, decltype(pw)::value>), grid, blk, lds, s, a,
                       o, ny);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (!fullg) {
    chi0 ? go(T_{}, F_{}, F_{}) : go(F_{}, F_{}, F_{});
  } else if (pwrite) {
    chi0 ? go(T_{}, T_{}, T_{}) : go(F_{}, T_{}, T_{});
  } else {
    chi0 ? go(T_{}, T_{}, F_{}) : go(F_{}, T_{}, F_{});
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

inline int launch_padj(int ny, const YArgs& a, const Optics& o, bool fullg, hipStream_t s) {
  const int w = pruned_waves(ny, true);
  const size_t lds = (size_t)w * pruned_wave_lds(ny, true);
  const dim3 grid = pruned_grid(a.nx, a.ngroups, w), blk(64 * w);
  STEM_TRACE(fullg ? "ssb_gadjoint" : "ssb_adjoint_pruned", s);
  if (fullg)
    hipLaunchKernelGGL(k_padj<true>, grid, blk, lds, s, a, o, ny);
  else
    hipLaunchKernelGGL(k_padj<false>, grid, blk, lds, s, a, o, ny);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem
