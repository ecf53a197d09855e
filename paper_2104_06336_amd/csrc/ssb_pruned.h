// Eq. 3 and its adjoint from the stored double-overlap values of G (the pruned array whose layout
// ssb_fused.h describes): the refocus sum of Sec. IV (only the summation runs again) and the
// adjoint without any transform.
//
// Work unit: the run of one pixel in one scan-frequency column mx (Qx = ix(mx) sx, mx in [0, Nx)),
// its stored values contiguous.  A wave gathers the descriptors of up to 64 runs at a time into
// lane registers (start and length, the set's first row frequency and hole, Kc and the phase
// polynomial of the column), then streams the runs in rounds of 64 lanes x 4 entries (coalesced
// loads) with the next rounds' loads in flight while one is summed, and adds every value, times
// its phase factor, into the column's T in LDS (one slot per row frequency my: the entries of a
// round have distinct my, so no two lanes touch one slot).
//
// Refocus (k_psum_stream) and adjoint (k_padj_stream) over the stored array: the columns are cut
// into pieces of equal cost, one wave each, as many as the GPU holds at once (tables built at
// FINALIZE, k_stream_*).  A piece's partial T is one row of the partial buffer; the phase pass
// adds a column's rows in order.
//
// The other scan lengths (k_psum, k_padj with FULLG): the runs are read from a block of full
// half-spectrum columns of G (pixel kd's column c at X + ((kd - xk0) (Nx/2+1) + c) Ny; a column
// mx > Nx/2 is the conjugate of column Nx - mx at -my), chunk by chunk of pixels; a wave (refocus)
// or workgroup (adjoint) owns a column and a pixel group, its partial T going to part[g]
// (column-major [mx][my]).  With PWRITE the values read are also stored as the pruned array.
#pragma once

#include "ssb_fused.h"

namespace stem {

struct RunDesc {
  int64_t e0;     // first entry of the run
  int32_t len;    // entries (0: the pixel has no pair in this column)
  int32_t a0;     // signed row frequency of the first entry
  int32_t split;  // entries before the hole of the set
  int32_t hl;     // hole length (0: none)
  int32_t lo;     // first entry of the run taken (entries [lo, len) are summed)
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
#ifndef STEM_ADJ_DEPTH
#define STEM_ADJ_DEPTH 3
#endif
constexpr int kAdjDepth = STEM_ADJ_DEPTH;  // rounds in flight per wave, adjoint

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
  RunDesc d{0, 0, 0, 0, 0, 0, 0.0, 0.0, ChiRow{0.0, 0.0, 0.0, 0.0, 0.0}};
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
    r.lo = rl(d.lo, j);
    return r;
  }
  __device__ __forceinline__ int lo(int j) const { return rl(d.lo, j); }
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
  return RunBatch{d, (uint64_t)__ballot(d.len > d.lo), nb};
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
  const int j = rb.next(r.j);
  return Round{j, j < rb.nb ? rb.lo(j) : 0};
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

// Adds the runs of a batch (pixels kb + j, column mx), times their phase factors, into the wave's
// column t of T.  CHI0: every phase factor is exactly 1.  The rounds go through kSumDepth register
// slots: slot d is summed, then refilled with the next round's loads, so kSumDepth - 1 rounds are
// in flight while one is summed.  A round's slices of 64 entries with no entry of the run are
// skipped (a wave-uniform test); inside a slice every lane works, and the lanes past the run's end
// read and write the wave's spare LDS slot t[ny], so the LDS accesses of a round issue back to back
// with no divergent branch between them.  Returns the pairs added.
template <bool CHI0, bool FULLG, bool PWRITE>
__device__ __forceinline__ unsigned long long sum_batch(const YArgs& a, const RunBatch& rb, int kb, int mx, int ny,
                                                        int lane, float2* t) {
  constexpr int D = kSumDepth;
  const int nb = rb.nb;
  unsigned long long cnt = 0;
  const int j0 = rb.next(-1);
  if (j0 >= nb) return 0;
  Round pos[D];
  float2 buf[D][4];
  const Round r0{j0, rb.lo(j0)};
  RoundCursor it{r0, r0};
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
        if (u0 == r.lo) cnt += (unsigned long long)(r.len - r.lo);
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
  return cnt;
}

// T of column mx over the pixels of group g (the sums of the scan lengths the fused kernels do not
// take, from full columns of G, chunk by chunk): the partial T of the group goes to part[g]
// (column-major [mx][my], summed by the phase pass like the fused sum's).
template <bool CHI0, bool FULLG, bool PWRITE>
__global__ void __launch_bounds__(64 * kPrunedCols) k_psum(YArgs a, Optics o, int ny) {
  if (state_unready(a)) return;
  extern __shared__ __align__(16) unsigned char s_dyn[];
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
    cnt += sum_batch<CHI0, FULLG, PWRITE>(a, rb, kb, mx, ny, lane, t);
  }
  float2* pgp = a.part + (int64_t)g * nx * ny + (int64_t)mx * ny;
  for (int i = lane; i < ny; i += 64) pgp[i] = a.accumulate ? cadd(pgp[i], t[i]) : t[i];
  unsigned long long cc = cnt + (cnt << kLoadShift);  // one 8-byte load per pair
  if (lane == 0) a.wcnt[wid] = a.accumulate ? a.wcnt[wid] + cc : cc;
}

// Refocus sum in balanced pieces.  The pruned array is column-major (the runs of a column's pixels
// follow one another), so a column's values are one contiguous stretch.  Each column is cut into
// pieces of equal cost, cost = entries + kRunCost per run with entries (a run costs at least one
// round whatever its length), the cost per piece Cc the same for every column (about total cost /
// nws, see k_stream_cands); one wave sums one piece.  Every wave thus does about the same work (a column of few
// pairs is one short piece), and no wave leaves its column: its partial T is one row of ny values
// at part + w ny, the pieces of column mx being the waves colseg[mx] .. colseg[mx + 1] - 1, which
// the phase pass adds in order.
constexpr int64_t kRunCost = 192;

// Per piece (tables from k_stream_*): the run (mx n_k + kd) holding its first entry, its entries
// [E0, E1) of the array, and for the adjoint the whole runs [ra, rb) whose first entry lies in
// [E0, E1) (the column's first piece from the column's first run, the last to its last, so that
// the pieces of a column take each of its runs once, empty ones included).  Tables built at
// FINALIZE: the column costs and spans by k_prune_runs, then k_stream_cands, k_stream_colseg and
// k_stream_waves.
struct PieceTab {
  int64_t run, e0, e1, ra, rb;
};

// Table of the columns, ctab (int64): colseg [nx + 1], then the cost per piece, then per column
// its cost and the span [first, last + 1) of its runs with entries (run indices), [nx][3], then
// the candidate costs per piece and their piece counts [kStreamCands][2].
constexpr int kStreamCands = 256;
__host__ __device__ inline size_t stream_ctab_words(int nx) {
  return (size_t)(nx + 1) + 1 + 3 * (size_t)nx + 2 * kStreamCands;
}

template <bool CHI0>
__global__ void __launch_bounds__(64 * kPrunedCols) k_psum_stream(YArgs a, Optics o, int ny, int nwmax,
                                                                  const PieceTab* __restrict__ wtab,
                                                                  const int64_t* __restrict__ ctab) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2* t = (float2*)(s_dyn + (size_t)wave * pruned_wave_lds(ny));
  if (state_unready(a)) return;
  const int nx = a.nx, n_k = a.n_k, nc = nx / 2 + 1;
  const int64_t wid = (int64_t)blockIdx.x * W + wave;
  if (wid >= nwmax || wid >= ctab[nx]) {
    if (lane == 0 && wid < nwmax) a.wcnt[wid] = 0ull;
    return;
  }
  const PieceTab pc = wtab[wid];
  // tables outside their ranges read nothing: the piece adds 0
  if (!(pc.run >= 0 && pc.run < (int64_t)nx * n_k && pc.e0 >= 0 && pc.e0 <= pc.e1 && pc.e1 <= a.pcap)) {
    for (int k = lane; k < ny; k += 64) a.part[wid * ny + k] = make_float2(0.f, 0.f);
    if (lane == 0) a.wcnt[wid] = 0ull;
    return;
  }
  const int64_t E0 = pc.e0, E1 = pc.e1;
  int64_t i = pc.run;
  const int mx = (int)(i / n_k);
  const int64_t cend =
      min(max(ctab[(nx + 2) + 3 * (int64_t)mx + 2], i + 1), (int64_t)(mx + 1) * n_k);  // within the column
  const bool mir = 2 * mx > nx;
  const int c = mir ? nx - mx : mx;
  double qx = 0.0;
  if (!CHI0) qx = (double)signed_index(mx, nx) * o.sx;
  for (int k = lane; k < ny; k += 64) t[k] = make_float2(0.f, 0.f);
  unsigned long long cnt = 0;
  while (true) {
    // runs [i, i + nb) of column mx, clipped to the piece
    const int nb = (int)min((int64_t)64, cend - i);
    RunDesc d{0, 0, 0, 0, 0, 0, 0.0, 0.0, ChiRow{0.0, 0.0, 0.0, 0.0, 0.0}};
    int64_t e1raw = 0;
    if (lane < nb) {
      const int kd = (int)(i + lane - (int64_t)mx * n_k);
      ColSet sd, sm;
      load_colsets(a.cst, (int64_t)kd * nc + c, sd, sm);
      const ColSet st = mir ? sm : sd;
      const int h0 = max(st.a0, st.b0), h1 = min(st.a1, st.b1);
      const int64_t e0 = a.poff[i + lane], e1 = a.poff[i + lane + 1];
      e1raw = e1;
      if (e0 >= 0 && e1 >= e0 && e1 <= a.pcap) {
        const int64_t b0 = min(max(e0, E0), e1);  // the run's entries inside the piece: [b0, b1)
        d.e0 = e0;
        d.lo = (int)(b0 - e0);
        d.len = (int)(max(min(e1, E1), b0) - e0);
      }
      d.a0 = st.a0;
      d.hl = h0 <= h1 ? h1 - h0 + 1 : 0;
      d.split = h0 - st.a0;
      if (!CHI0) {
        const double2 k = a.kc[kd];
        const double kch = chi_poly(k.x, k.y, o) + (a.theta ? (double)a.theta[kd] : 0.0);
        d.ch = chi_row(chi_column(o.lk * (k.x - qx), o), o.lk * k.y, -o.lk * o.sy, kch);
      }
    }
    const RunBatch rb = make_batch(d, nb);
    cnt += sum_batch<CHI0, false, false>(a, rb, 0, mx, ny, lane, t);
    i += nb;
    if (RunBatch::rl64(e1raw, nb - 1) >= E1 || i >= cend) break;
  }
  float2* dst = a.part + wid * ny;
  for (int k = lane; k < ny; k += 64) dst[k] = t[k];
  unsigned long long cc = cnt + (cnt << kLoadShift);  // one 8-byte load per pair
  if (lane == 0) a.wcnt[wid] = cc;
}

// The cost of the runs [r0, r0 + n) of the array (offsets poff): entries + kRunCost per non-empty run.
__device__ __forceinline__ int64_t runs_cost(const int64_t* __restrict__ poff, int64_t r0, int n) {
  int64_t c = 0;
  for (int k = 0; k < n; ++k) {
    const int64_t len = poff[r0 + k + 1] - poff[r0 + k];
    c += len > 0 ? len + kRunCost : 0;
  }
  return c;
}

// The sum of the column costs, by every thread of a workgroup.
__device__ __forceinline__ int64_t stream_total_cost(int nx, const int64_t* __restrict__ col, int64_t* s_sum) {
  int64_t tot = 0;
  for (int mx = threadIdx.x; mx < nx; mx += 256) tot += col[3 * mx];
  s_sum[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  const int64_t total = s_sum[0];
  __syncthreads();
  return total;
}

// Candidate t (workgroup t of kStreamCands) for the cost per piece: lo + t (hi - lo) / (kStreamCands
// - 1) over [lo, hi] = [total / nws, total / (nws - nx)] (the second always gives at most nws
// pieces, as the pieces number at most total / Cc + nx), and its number of pieces.
__global__ void __launch_bounds__(256) k_stream_cands(int nx, int nws, int64_t* __restrict__ ctab) {
  __shared__ int64_t s_sum[256];
  const int64_t* col = ctab + (nx + 2);
  const int64_t total = stream_total_cost(nx, col, s_sum);
  const int64_t lo = total > 0 ? (total + nws - 1) / nws : 1;
  const int64_t hi = total <= 0 ? 1 : nws > nx ? (total + (nws - nx) - 1) / (nws - nx) : total;
  const int64_t c = hi > lo ? lo + (int64_t)blockIdx.x * (hi - lo) / (kStreamCands - 1) : hi;
  int64_t n = 0;
  for (int mx = threadIdx.x; mx < nx; mx += 256) n += (col[3 * mx] + c - 1) / c;
  s_sum[threadIdx.x] = n;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int64_t* cand = ctab + (nx + 2) + 3 * (int64_t)nx;
    cand[2 * blockIdx.x] = c;
    cand[2 * blockIdx.x + 1] = s_sum[0];
  }
}

// One workgroup: the cost per piece Cc, the smallest candidate whose pieces number at most nws (the
// last candidate always does), so that the launch's nws waves (the waves the GPU holds at once)
// each sum one piece and every compute unit gets the same work; then colseg, the exclusive scan of
// the pieces per column ceil(cost / Cc).
__global__ void __launch_bounds__(256) k_stream_colseg(int nx, int nws, int64_t* __restrict__ ctab) {
  __shared__ int64_t s_sum[256];
  const int64_t* col = ctab + (nx + 2);
  const int64_t* cand = col + 3 * (int64_t)nx;
  static_assert(kStreamCands == 256, "one candidate per thread");
  const int t = threadIdx.x;
  s_sum[t] = cand[2 * t + 1] <= nws || t == kStreamCands - 1 ? cand[2 * t] : INT64_MAX;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) s_sum[t] = min(s_sum[t], s_sum[t + off]);
    __syncthreads();
  }
  const int64_t Cc = s_sum[0];
  __syncthreads();
  const int per = (nx + 255) / 256, m0 = t * per;
  int64_t n = 0;
  for (int mx = m0; mx < m0 + per && mx < nx; ++mx) n += (col[3 * mx] + Cc - 1) / Cc;
  s_sum[t] = n;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t v = t >= off ? s_sum[t - off] : 0;
    __syncthreads();
    s_sum[t] += v;
    __syncthreads();
  }
  int64_t base = s_sum[t] - n;
  for (int mx = m0; mx < m0 + per && mx < nx; ++mx) {
    ctab[mx] = base;
    base += (col[3 * mx] + Cc - 1) / Cc;
  }
  if (t == 255) {
    ctab[nx] = s_sum[255];
    ctab[nx + 1] = Cc;
  }
}

// Per column (workgroup): the pieces' first runs, entry ranges and (after a barrier) run ranges.  Piece p of column mx starts at
// cost p Cc of the column; inside run r (cost [c_r, c_r + kRunCost + len)) that is entry
// max(0, p Cc - c_r - kRunCost) of the run.  Piece p ends where piece p + 1 starts, the last at
// the column's end.
__global__ void __launch_bounds__(256) k_stream_waves(int n_k, const int64_t* __restrict__ poff, int nx,
                                                      const int64_t* __restrict__ ctab, PieceTab* __restrict__ wtab) {
  __shared__ int64_t s_pre[256];
  const int mx = blockIdx.x;
  const int64_t* col = ctab + (nx + 2) + 3 * (int64_t)mx;
  const int64_t ccost = col[0], Cc = ctab[nx + 1], seg0 = ctab[mx];
  if (ccost == 0) return;
  const int64_t npieces = (ccost + Cc - 1) / Cc;
  const int q = (n_k + 255) / 256, k0 = min((int)threadIdx.x * q, n_k), k1 = min(k0 + q, n_k);
  const int64_t r0 = (int64_t)mx * n_k;
  const int64_t mine = runs_cost(poff, r0 + k0, k1 - k0);
  s_pre[threadIdx.x] = mine;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t v = threadIdx.x >= off ? s_pre[threadIdx.x - off] : 0;
    __syncthreads();
    s_pre[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t cr = s_pre[threadIdx.x] - mine;  // cost before this thread's first run
  for (int kd = k0; kd < k1; ++kd) {
    const int64_t e0 = poff[r0 + kd], len = poff[r0 + kd + 1] - e0;
    if (len <= 0) continue;
    const int64_t c1 = cr + kRunCost + len;
    // the pieces starting inside this run's cost range [cr, c1)
    for (int64_t p = (cr + Cc - 1) / Cc; p < npieces && p * Cc < c1; ++p) {
      const int64_t e = e0 + max((int64_t)0, p * Cc - cr - kRunCost);
      wtab[seg0 + p].run = r0 + kd;
      wtab[seg0 + p].e0 = e;
      if (p > 0) wtab[seg0 + p - 1].e1 = e;
    }
    cr = c1;
  }
  if (threadIdx.x == 255) {
    const int64_t ce = mx + 1 < nx ? poff[r0 + n_k] : poff[(int64_t)nx * n_k];
    wtab[seg0 + npieces - 1].e1 = ce;
  }
  __syncthreads();
  // the adjoint's run ranges: piece p takes the runs whose first entry lies in its entries (the
  // first piece from the column's first run, the last to its last run)
  auto first_run = [&](const PieceTab& q) { return q.e0 == poff[q.run] ? q.run : q.run + 1; };
  for (int64_t p = threadIdx.x; p < npieces; p += 256) {
    wtab[seg0 + p].ra = p == 0 ? r0 : first_run(wtab[seg0 + p]);
    wtab[seg0 + p].rb = p + 1 == npieces ? r0 + n_k : first_run(wtab[seg0 + p + 1]);
  }
}

// FP64 sum over the 64 lanes of a wave (every lane active), returned to every lane
__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Adds the adjoint terms of a batch's runs (pixels kd0 + stride j, column mx) to dc and returns
// on lane j -(sum of w) of run j (0 without pairs).  tb: the column of Tbar in LDS.  Rounds are
// pipelined through kAdjDepth register slots as in sum_batch; the moments of a run carry over its
// consecutive rounds.
template <bool FULLG>
__device__ __forceinline__ float adj_batch(const YArgs& a, const Optics& o, const RunBatch& rb, int kd0, int stride,
                                           int mx, int ny, int lane, const float2* tb, double qx, double s2pi,
                                           double* dc) {
  constexpr int D = kAdjDepth;
  const int nb = rb.nb;
  float wth = 0.f;
  const int j0 = rb.next(-1);
  Round pos[D];
  float2 buf[D][4];
  RoundCursor it{Round{j0, 0}, Round{j0, 0}};
  if (j0 < nb) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const Round l = it.load_target(nb);
      load_round<FULLG>(a, rb.at(l.j), kd0 + stride * l.j, mx, ny, l.u0, lane, buf[d]);
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
      load_round<FULLG>(a, rb.at(l.j), kd0 + stride * l.j, mx, ny, l.u0, lane, buf[d]);
      pos[d] = it.take(rb);
    }
  }
  return wth;
}

// Adjoint of Eq. 3 from the stored values: for every pair, z = G e^{i psi}, w = Re(conj(Tbar(Q)) i z);
// per (pixel, column) run the moments M_n = sum w wy^n (n = 0..4) give the eight dL/dc terms (the
// B_j(K - Q) are polynomials in wy along a column, see k_yadjoint); dL/dtheta[kd] = -sum w.
// Over full columns of G (the other scan lengths): a workgroup owns a column and a pixel group whose
// pixels its waves share out (wave w takes every W-th pixel), the column of Tbar loaded into LDS
// once.  Partials: pdc[workgroup][8] (FP64), pdth[mx][kd] (FP32; one writer per entry), the
// workgroup's four waves combined into one dL/dc partial.
template <bool FULLG>
__global__ void __launch_bounds__(64 * kAdjWaves) k_padj(YArgs a, Optics o, int ny) {
  if (state_unready(a)) return;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  constexpr int W = kAdjWaves;
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
    const float wth = adj_batch<FULLG>(a, o, rb, kd0, W, mx, ny, lane, tb, qx, s2pi, dc);
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

// Adjoint over the stored values in the refocus sum's pieces: the wave of piece w takes the whole
// runs [ra, rb) of its column (no run is split, so dL/dtheta[mx][kd] keeps one writer; runs
// outside the column's span of runs with pairs get 0 without a gather), with its own copy of the
// column of Tbar in LDS; dL/dc: one partial per wave, pdc[w][8].
__global__ void __launch_bounds__(64 * kPrunedCols) k_padj_stream(YArgs a, Optics o, int ny, int nwmax,
                                                                  const PieceTab* __restrict__ wtab,
                                                                  const int64_t* __restrict__ ctab) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  const int W = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2* tb = (float2*)(s_dyn + (size_t)wave * padj_block_lds(ny));
  if (state_unready(a)) return;
  const int nx = a.nx, n_k = a.n_k;
  const int64_t wid = (int64_t)blockIdx.x * W + wave;
  if (wid >= nwmax) return;
  if (wid >= ctab[nx]) {
    if (lane < 8) a.pdc[wid * 8 + lane] = 0.0;
    return;
  }
  const PieceTab pc = wtab[wid];
  // tables outside their ranges read nothing
  if (!(pc.run >= 0 && pc.run < (int64_t)nx * n_k)) {
    if (lane < 8) a.pdc[wid * 8 + lane] = 0.0;
    return;
  }
  const int mx = (int)(pc.run / n_k);
  const int64_t c0 = (int64_t)mx * n_k;
  const int64_t* col = ctab + (nx + 2) + 3 * (int64_t)mx;
  const int64_t ra = min(max(pc.ra, c0), c0 + n_k), rb = min(max(pc.rb, ra), c0 + n_k);
  const int64_t ga = min(max(col[1], ra), rb), gb = min(max(col[2], ga), rb);
  float* pth = a.pdth + c0;
  for (int64_t r = ra + lane; r < rb; r += 64)
    if (r < ga || r >= gb) pth[r - c0] = 0.f;
  for (int i = lane; i < ny; i += 64) tb[i] = a.Tbt[(int64_t)mx * ny + i];
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const double s2pi = 6.283185307179586476925286766559 / o.lam;
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  for (int64_t i = ga; i < gb; i += 64) {
    const int kd0 = (int)(i - c0);
    const int nb = (int)min((int64_t)64, gb - i);
    const RunBatch rb = make_batch(gather_run(a, o, kd0, 1, nb, mx, lane, true, false), nb);
    const float wth = adj_batch<false>(a, o, rb, kd0, 1, mx, ny, lane, tb, qx, s2pi, dc);
    if (lane < nb) pth[kd0 + lane] = wth;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double t = wave_sum_f64(dc[j]);
    if (lane == 0) a.pdc[wid * 8 + j] = t;
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

// the sums of the other scan lengths over full columns of G at a.X (pixels from a.xk0), chunk by
// chunk; pwrite: also store the values as the pruned array
inline int launch_psum(int ny, const YArgs& a, const Optics& o, int chi0, bool pwrite, hipStream_t s) {
  const int w = psum_waves(ny);
  const size_t lds = (size_t)w * pruned_wave_lds(ny);
  const dim3 grid((unsigned)(psum_launch_waves(ny, a.nx, a.ngroups) / w)), blk(64 * w);
  STEM_TRACE("ssb_gsum", s);
  auto go = [&](auto c0, auto pw) {
    hipLaunchKernelGGL((k_psum<decltype(c0)::value, true, decltype(pw)::value>), grid, blk, lds, s, a, o, ny);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (pwrite)
    chi0 ? go(T_{}, T_{}) : go(F_{}, T_{});
  else
    chi0 ? go(T_{}, F_{}) : go(F_{}, F_{});
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// Waves of the refocus sum in balanced pieces: the waves MI355X holds at once (256 compute units;
// per unit the workgroups its 160 KB of LDS holds, at most 5 waves per SIMD by registers), so
// that all of them run together and every unit gets the same number of pieces.
inline int64_t psum_stream_waves(int ny) {
  const int w = psum_waves(ny);
  const int64_t per_cu = (int64_t)((160u << 10) / ((size_t)w * pruned_wave_lds(ny))) * w;
  return 256 * (per_cu < 20 ? per_cu : 20);
}

// the refocus sum over the stored values in balanced pieces: nwmax waves at most
inline int launch_psum_stream(int ny, const YArgs& a, const Optics& o, int chi0, int nwmax, const PieceTab* wtab,
                              const int64_t* ctab, hipStream_t s) {
  const int w = psum_waves(ny);
  const size_t lds = (size_t)w * pruned_wave_lds(ny);
  const dim3 grid((unsigned)((nwmax + w - 1) / w)), blk(64 * w);
  STEM_TRACE("ssb_reduce", s);
  if (chi0)
    hipLaunchKernelGGL(k_psum_stream<true>, grid, blk, lds, s, a, o, ny, nwmax, wtab, ctab);
  else
    hipLaunchKernelGGL(k_psum_stream<false>, grid, blk, lds, s, a, o, ny, nwmax, wtab, ctab);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// the adjoint over the stored values in the refocus sum's pieces
inline int launch_padj_stream(int ny, const YArgs& a, const Optics& o, int nwmax, const PieceTab* wtab,
                              const int64_t* ctab, hipStream_t s) {
  const int w = psum_waves(ny);
  const size_t lds = (size_t)w * padj_block_lds(ny);
  const dim3 grid((unsigned)((nwmax + w - 1) / w)), blk(64 * w);
  STEM_TRACE("ssb_adjoint_pruned", s);
  hipLaunchKernelGGL(k_padj_stream, grid, blk, lds, s, a, o, ny, nwmax, wtab, ctab);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// the adjoint of the other scan lengths over full columns of G at a.X, chunk by chunk
inline int launch_padj(int ny, const YArgs& a, const Optics& o, hipStream_t s) {
  const size_t lds = padj_block_lds(ny);
  const dim3 grid((unsigned)padj_partials(a.nx, a.ngroups)), blk(64 * kAdjWaves);
  STEM_TRACE("ssb_gadjoint", s);
  hipLaunchKernelGGL(k_padj<true>, grid, blk, lds, s, a, o, ny);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem
