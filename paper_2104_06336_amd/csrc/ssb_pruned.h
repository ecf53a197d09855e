// Eq. 3 and its adjoint from the stored double-overlap values of G (the pruned array whose layout
// ssb_fused.h describes): the refocus sum of Sec. IV (only the summation runs again) and the
// adjoint without any transform.
//
// Refocus sum: a wave owns one scan-frequency column mx of the whole plane (Qx = ix(mx) sx, mx in
// [0, Nx)) and a group of pixels, and keeps the column's T in LDS.  The lanes first gather the
// descriptors of 64 pixels at a time (start and length of the pixel's run for this column, the
// set's first row frequency and hole, Kc and chi(Kc) + theta) into LDS; the wave then streams the
// runs of stored values in rounds of 64 lanes x 4 entries (contiguous, coalesced loads), with the
// loads of the next rounds in flight while one is summed, and adds every value, times its phase
// factor, into T (one slot per row frequency my: the entries of a round have distinct my, so no
// two lanes touch one slot).  The partial T of the group goes to part[g] (column-major [mx][my],
// summed by the phase pass like the fused sum's).
//
// Adjoint: a workgroup owns a column and a pixel group whose pixels its waves share out (wave w
// takes every W-th pixel); the column of Tbar is loaded into LDS once per workgroup.
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
  double kx, ky;  // Kc
  ChiRow ch;      // the phase of the pixel's pairs in this column, in revolutions, by row index
};

// columns (waves) per workgroup of the refocus sum (fewer while its LDS would pass 64 KB), and
// waves per workgroup of the adjoint
#ifndef STEM_PRUNED_COLS
#define STEM_PRUNED_COLS 4
#endif
constexpr int kPrunedCols = STEM_PRUNED_COLS;
constexpr int kAdjWaves = 4;
#ifndef STEM_SUM_DEPTH
#define STEM_SUM_DEPTH 4
#endif
constexpr int kSumDepth = STEM_SUM_DEPTH;  // rounds in flight per wave, refocus sum
constexpr int kAdjDepth = 3;     // rounds in flight per wave, adjoint

// LDS bytes of one refocus wave: its column of T and a spare slot (the target of the lanes past a
// run's end), padded to 16 bytes
__host__ __device__ inline size_t pruned_wave_lds(int ny) { return (size_t)(ny + 2) * sizeof(float2); }

// LDS bytes of an adjoint workgroup: its column of Tbar
__host__ __device__ inline size_t padj_block_lds(int ny) { return (size_t)ny * sizeof(float2); }

// descriptors of the pixels kd0 + lane * stride (lane < nb) for column mx; fullg: run lengths from
// the sets (e0 = the pruned array's offset when it exists); general: Kc and the phase polynomial
// of the column (chi(Kc) + theta evaluated from Kc and theta when a.kch_inline)
__device__ __forceinline__ RunDesc gather_run(const YArgs& a, const Optics& o, int kd0, int stride, int nb, int mx,
                                              int lane, bool general, bool fullg) {
  const int nx = a.nx, nc = nx / 2 + 1;
  const bool mir = 2 * mx > nx;
  const int c = mir ? nx - mx : mx;
  RunDesc d{0, 0, 0, 0, 0, 0.0, 0.0, ChiRow{0.0, 0.0, 0.0, 0.0, 0.0}};
  if (lane < nb) {
    const int kd = kd0 + lane * stride;
    ColSet sd, sm;
    load_colsets(a.cst, (int64_t)kd * nc + c, sd, sm);
    const ColSet s = mir ? sm : sd;
    const int h0 = max(s.a0, s.b0), h1 = min(s.a1, s.b1);
    if (fullg) {
      d.e0 = a.poff ? a.poff[(int64_t)mx * a.n_k + kd] : 0;
      d.len = set_size(s);
    } else {
      const int64_t e0 = a.poff[(int64_t)mx * a.n_k + kd], e1 = a.poff[(int64_t)mx * a.n_k + kd + 1];
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
      const double kch =
          a.kch_inline ? chi_poly(k.x, k.y, o) + (a.theta ? (double)a.theta[kd] : 0.0) : a.kchi[kd];
      const double qx = (double)signed_index(mx, nx) * o.sx;
      d.ch = chi_row(chi_column(o.lk * (k.x - qx), o), o.lk * k.y, -o.lk * o.sy, kch);
    }
  }
  return d;
}

// A batch of up to 64 runs held in registers: lane j keeps run j's descriptor; the wave reads run
// j's fields with readlane (uniform j) and walks the non-empty runs through a ballot mask.
struct RunBatch {
  RunDesc d;
  uint64_t mask;  // bit j: run j has entries
  int nb;

  __device__ __forceinline__ static int rl(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
  __device__ __forceinline__ static int64_t rl64(int64_t v, int j) {
    const uint32_t lo = (uint32_t)rl((int)(uint32_t)v, j), hi = (uint32_t)rl((int)(v >> 32), j);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  }
  __device__ __forceinline__ static double rld(double v, int j) { return __longlong_as_double(rl64(__double_as_longlong(v), j)); }

  __device__ __forceinline__ int len(int j) const { return rl(d.len, j); }
  // run j's extent (the entries and their row frequencies)
  __device__ __forceinline__ RunDesc at(int j) const {
    RunDesc r;
    r.e0 = rl64(d.e0, j);
    r.len = rl(d.len, j);
    r.a0 = rl(d.a0, j);
    r.split = rl(d.split, j);
    r.hl = rl(d.hl, j);
    return r;
  }
  __device__ __forceinline__ ChiRow chi(int j) const {
    return ChiRow{rld(d.ch.p0, j), rld(d.ch.p1, j), rld(d.ch.p2, j), rld(d.ch.p3, j), rld(d.ch.p4, j)};
  }
  __device__ __forceinline__ double2 kc(int j) const { return make_double2(rld(d.kx, j), rld(d.ky, j)); }
  // the first run with entries after slot j (nb if none)
  __device__ __forceinline__ int next(int j) const {
    const uint64_t m = j >= 63 ? 0ull : mask & (~0ull << (j + 1));
    return m ? __builtin_ctzll(m) : nb;
  }
};

__device__ __forceinline__ RunBatch make_batch(const RunDesc& d, int nb) {
  return RunBatch{d, (uint64_t)__ballot(d.len > 0), nb};
}

// Signed row frequency of entry u of run r.
__device__ __forceinline__ int run_iy(const RunDesc& r, int u) { return r.a0 + u + ((r.hl && u >= r.split) ? r.hl : 0); }

// One round of a non-empty run: entries u0 + lane + 64 q (q < 4) of run r of pixel kd, column mx,
// from the pruned array or (FULLG) from the full columns of G.  Every lane loads (past the run's
// end it reloads its last entry, zeroed after the load), so the loads are not under divergent
// control flow and stay in flight while earlier rounds are summed.
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
    const int uc = min(u, r.len - 1);
    float2 x;
    if constexpr (FULLG) {
      const int iy = run_iy(r, uc);
      const int my = iy < 0 ? iy + ny : iy;
      x = mir ? cconj(col[(ny - my) % ny]) : col[my];
    } else {
      x = a.pg[r.e0 + uc];
    }
    gv[q] = x;
  }
}

// A round: entries [u0, u0 + 256) of run j of the batch (j == nb: none).
struct Round {
  int j, u0;
};

__device__ __forceinline__ Round next_round(const RunBatch& rb, Round r) {
  if (r.j >= rb.nb) return r;
  if (r.u0 + 256 < rb.len(r.j)) return Round{r.j, r.u0 + 256};
  return Round{rb.next(r.j), 0};
}

// The rounds of a batch in order.  `at` is the next round to load; `safe` the last real one, whose
// entries are loaded again (and ignored) once the rounds run out, so that every load of the
// pipelined loops is unconditional and inside the arrays.
struct RoundCursor {
  Round at, safe;
  __device__ __forceinline__ Round take(const RunBatch& rb) {
    const Round r = at;
    if (at.j < rb.nb) safe = at;
    at = next_round(rb, at);
    return r;
  }
  __device__ __forceinline__ Round load_target(int nb) const { return at.j < nb ? at : safe; }
};

// A wave's or workgroup's work: column mx and the pixels [kd_a, kd_b) of its group g.
struct PrunedItem {
  int mx, g, kd_a, kd_b;
  bool live;
};

// The work of wave w of workgroup blk: the pixels [kd_a, kd_b) of group g = blk % ngroups of
// ngroups equal shares of [k0, k1), and column mx = (blk / ngroups) W + w (W = 1 for the adjoint,
// whose workgroup takes one column).  In the column-major pruned array the runs of a column's
// pixels follow one another, so each item reads one contiguous stretch.
__device__ __forceinline__ PrunedItem pruned_item(const YArgs& a, int64_t blk, int w, int W) {
  PrunedItem it{0, 0, 0, 0, false};
  it.g = (int)(blk % a.ngroups);
  it.mx = (int)(blk / a.ngroups) * W + w;
  if (it.mx >= a.nx) return it;
  it.kd_a = a.k0 + (int)((int64_t)(a.k1 - a.k0) * it.g / a.ngroups);
  it.kd_b = a.k0 + (int)((int64_t)(a.k1 - a.k0) * (it.g + 1) / a.ngroups);
  it.live = true;
  return it;
}

// The share of wave w of W in the pixels [kd_a, kd_b): kd = kd_a + w + W i, i < count.
struct WavePixels {
  int kd_a, count;
};

__device__ __forceinline__ WavePixels wave_pixels(int kd_a, int kd_b, int w, int W) {
  const int n = kd_b - kd_a - w;
  return WavePixels{kd_a + w, n > 0 ? (n + W - 1) / W : 0};
}

// T of column mx over the pixels of group g from the stored values.  CHI0: every phase factor is
// exactly 1.  The rounds go through kSumDepth register slots: slot d is summed, then refilled
// with the next round's loads, so kSumDepth - 1 rounds are in flight while one is summed.  A
// round's slices of 64 entries with no entry of the run are skipped (a wave-uniform test); inside
// a slice every lane works, and the lanes past the run's end read and write the wave's spare LDS
// slot, so the LDS accesses of a round issue back to back with no divergent branch between them.
template <bool CHI0, bool FULLG, bool PWRITE>
__global__ void __launch_bounds__(64 * kPrunedCols) k_psum(YArgs a, Optics o, int ny) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  constexpr int D = kSumDepth;
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2* t = (float2*)(s_dyn + (size_t)wave * pruned_wave_lds(ny));
  const int nx = a.nx;
  const int64_t wid = (int64_t)blockIdx.x * W + wave;
  const PrunedItem pi = pruned_item(a, blockIdx.x, wave, W);
  if (!pi.live) {
    if (lane == 0 && !a.accumulate) a.wcnt[wid] = 0ull;
    return;
  }
  const int mx = pi.mx, g = pi.g;
  for (int i = lane; i < ny; i += 64) t[i] = make_float2(0.f, 0.f);
  const WavePixels wp = wave_pixels(pi.kd_a, pi.kd_b, 0, 1);
  unsigned long long cnt = 0;
  for (int i0 = 0; i0 < wp.count; i0 += 64) {
    const int kb = wp.kd_a + i0;
    const int nb = min(64, wp.count - i0);
    const RunBatch rb = make_batch(gather_run(a, o, kb, 1, nb, mx, lane, !CHI0, FULLG), nb);
    const int j0 = rb.next(-1);
    if (j0 >= nb) continue;
    Round pos[D];
    float2 buf[D][4];
    RoundCursor it{Round{j0, 0}, Round{j0, 0}};
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const Round l = it.load_target(nb);
      load_round<FULLG>(a, rb.at(l.j), kb + l.j, mx, ny, l.u0, lane, buf[d]);
      pos[d] = it.take(rb);
    }
    while (pos[0].j < nb) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (pos[d].j < nb) {
          const RunDesc r = rb.at(pos[d].j);
          const int u0 = pos[d].u0;
          if (u0 == 0) cnt += (unsigned long long)r.len;
          ChiRow ch{};
          if constexpr (!CHI0) ch = rb.chi(pos[d].j);
          int ad[4];
          float2 val[4], tv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int u = u0 + lane + 64 * q;
            const int iy = run_iy(r, u);
            ad[q] = u < r.len ? (iy < 0 ? iy + ny : iy) : ny;
            val[q] = buf[d][q];
            if (u0 + 64 * q < r.len) {
              if constexpr (PWRITE) {
                if (u < r.len && r.e0 + u < a.pcap) a.pgw[r.e0 + u] = val[q];
              }
              if constexpr (!CHI0) {
                const float2 e = expi_rev(chi_row_eval(ch, (double)iy));
                const float2 x = val[q];
                val[q] = make_float2(x.x * e.x - x.y * e.y, x.x * e.y + x.y * e.x);
              }
            }
          }
          // the entries of a round are distinct row frequencies of one run: read all, then write
#pragma unroll
          for (int q = 0; q < 4; ++q) tv[q] = t[ad[q]];
#pragma unroll
          for (int q = 0; q < 4; ++q) t[ad[q]] = cadd(tv[q], val[q]);
        }
        const Round l = it.load_target(nb);
        load_round<FULLG>(a, rb.at(l.j), kb + l.j, mx, ny, l.u0, lane, buf[d]);
        pos[d] = it.take(rb);
      }
    }
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
// Rounds are pipelined through kAdjDepth register slots as in k_psum; the moments of a run carry
// over its consecutive rounds.  Partials: pdc[workgroup][8] (FP64), pdth[mx][kd] (FP32; one writer per
// entry), the workgroup's four waves combined into one dL/dc partial.
template <bool FULLG>
__global__ void __launch_bounds__(64 * kAdjWaves) k_padj(YArgs a, Optics o, int ny) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  constexpr int D = kAdjDepth, W = kAdjWaves;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2* tb = (float2*)s_dyn;
  const int nx = a.nx;
  const PrunedItem pi = pruned_item(a, blockIdx.x, 0, 1);
  if (!pi.live) {
    if (wave == 0 && lane < 8 && !a.accumulate) a.pdc[(int64_t)blockIdx.x * 8 + lane] = 0.0;
    return;
  }
  const int mx = pi.mx;
  for (int i = threadIdx.x; i < ny; i += blockDim.x) tb[i] = a.Tbt[(int64_t)mx * ny + i];
  __syncthreads();
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const double s2pi = 6.283185307179586476925286766559 / o.lam;
  const WavePixels wp = wave_pixels(pi.kd_a, pi.kd_b, wave, W);
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  float* pth = a.pdth + (int64_t)mx * a.n_k;
  for (int i0 = 0; i0 < wp.count; i0 += 64) {
    const int kd0 = wp.kd_a + W * i0;
    const int nb = min(64, wp.count - i0);
    const RunBatch rb = make_batch(gather_run(a, o, kd0, W, nb, mx, lane, true, FULLG), nb);
    float wth = 0.f;  // lane j: -(sum of w) of pixel j of the batch (0 without pairs in this column)
    const int j0 = rb.next(-1);
    Round pos[D];
    float2 buf[D][4];
    RoundCursor it{Round{j0, 0}, Round{j0, 0}};
    if (j0 < nb) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const Round l = it.load_target(nb);
        load_round<FULLG>(a, rb.at(l.j), kd0 + W * l.j, mx, ny, l.u0, lane, buf[d]);
        pos[d] = it.take(rb);
      }
    } else {
      pos[0] = Round{nb, 0};
    }
    double M0 = 0.0, M1 = 0.0, M2 = 0.0, M3 = 0.0, M4 = 0.0;
    while (pos[0].j < nb) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (pos[d].j < nb) {
          const RunDesc r = rb.at(pos[d].j);
          const double2 kc = rb.kc(pos[d].j);
          const ChiRow ch = rb.chi(pos[d].j);
          const int u0 = pos[d].u0;
          const double wx = o.lk * (kc.x - qx);
          const double A = o.lk * kc.y, B = -o.lk * o.sy;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (u0 + 64 * q >= r.len) continue;  // wave-uniform: no entry of the run in this slice
            const int u = u0 + lane + 64 * q;
            const bool in = u < r.len;
            const int iy = run_iy(r, u);
            const int my = in ? (iy < 0 ? iy + ny : iy) : 0;
            const double ty = (double)iy;
            const double wy = fma(B, ty, A);
            const float2 e = expi_rev(chi_row_eval(ch, ty));
            const float2 gq = buf[d][q];
            const float2 z = make_float2(gq.x * e.x - gq.y * e.y, gq.x * e.y + gq.y * e.x);
            const float2 tq = tb[my];
            double t = in ? (double)(tq.x * (-z.y) + tq.y * z.x) : 0.0;
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
          if (u0 + 256 >= r.len) {
            // last round of the run: this lane's sum over its pairs of w B_j(K - Q), B_j as
            // polynomials in wy
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
              chi_basis(kc.x, kc.y, o, bk);
#pragma unroll
              for (int q = 0; q < 8; ++q) dc[q] -= bk[q] * wsum;
            }
            if (lane == pos[d].j) wth = (float)-wsum;
            M0 = M1 = M2 = M3 = M4 = 0.0;
          }
        }
        const Round l = it.load_target(nb);
        load_round<FULLG>(a, rb.at(l.j), kd0 + W * l.j, mx, ny, l.u0, lane, buf[d]);
        pos[d] = it.take(rb);
      }
    }
    if (lane < nb) pth[kd0 + W * lane] = wth;
  }
  // the workgroup's dL/dc: the waves' sums added in wave order
  __shared__ double s_dc[kAdjWaves][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double t = wave_sum_f64(dc[j]);
    if (lane == 0) s_dc[wave][j] = t;
  }
  __syncthreads();
  if (wave == 0 && lane < 8) {
    double t = s_dc[0][lane];
#pragma unroll
    for (int w = 1; w < kAdjWaves; ++w) t += s_dc[w][lane];
    double* p = a.pdc + (int64_t)blockIdx.x * 8 + lane;
    *p = a.accumulate ? *p + t : t;
  }
}

inline int psum_waves(int ny) {
  int w = kPrunedCols;
  while (w > 1 && (size_t)w * pruned_wave_lds(ny) > (64u << 10)) w >>= 1;
  return w;
}

// waves a launch writes partials for (wave index blockIdx.x * W + wave)
inline int64_t psum_launch_waves(int ny, int nx, int ngroups) {
  const int w = psum_waves(ny);
  return (int64_t)((nx + w - 1) / w) * ngroups * w;
}

// dL/dc partials of an adjoint launch over the stored values (one per workgroup)
inline int64_t padj_partials(int nx, int ngroups) { return (int64_t)nx * ngroups; }

// fullg: the runs from full columns of G at a.X (pixels from a.xk0); pwrite: also store the values
// as the pruned array
inline int launch_psum(int ny, const YArgs& a, const Optics& o, int chi0, bool fullg, bool pwrite, hipStream_t s) {
  const int w = psum_waves(ny);
  const size_t lds = (size_t)w * pruned_wave_lds(ny);
  const dim3 grid((unsigned)(psum_launch_waves(ny, a.nx, a.ngroups) / w)), blk(64 * w);
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
  const size_t lds = padj_block_lds(ny);
  const dim3 grid((unsigned)padj_partials(a.nx, a.ngroups)), blk(64 * kAdjWaves);
  STEM_TRACE(fullg ? "ssb_gadjoint" : "ssb_adjoint_pruned", s);
  if (fullg)
    hipLaunchKernelGGL(k_padj<true>, grid, blk, lds, s, a, o, ny);
  else
    hipLaunchKernelGGL(k_padj<false>, grid, blk, lds, s, a, o, ny);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem
