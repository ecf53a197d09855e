// Scan-DFT kernels of the SSB path (Eq. 2 fused with Eq. 3 and with its adjoint), templated on
// the transform along one scan axis: the FP32 Stockham FFT or the split-precision matrix-core
// DFT.  The FP32 launchers are instantiated with the host code; each split precision has a
// translation unit of its own.
#pragma once

#include <type_traits>

#include "common.h"
#include "fft_wave.h"
#include "geom.h"
#include "mfma_dft.h"
#include "optics.h"
#include "trace.h"

namespace stem {

constexpr int kXWaveStride = kFftLds + 4;
constexpr int kYThreads = 256;

// ---------------------------------------------------------------------------------------------
// Transforms of the scan DFT (Eq. 2) along one scan axis, per wavefront: 16 complex values per
// lane, B = 1024/N sequences of length N.  XfFft is the FP32 Stockham FFT; XfMfma the
// split-precision matrix-core DFT.  in()/out() give the (sequence, index) of each register;
// registers are grouped in "slots" that share one output sequence (column) for every lane.

template <int N_>
struct XfFft {
  static constexpr int N = N_;
  static constexpr bool kMfma = false;
  static constexpr int RL = fft_last_radix<N>();
  static constexpr int NB = N / RL;
  static constexpr bool kUniformCol = NB >= kWave;
  static constexpr int slot_of(int i) { return kUniformCol ? (kWave * (i / RL)) / NB : i / RL; }
  static constexpr int kSlots = slot_of(15) + 1;
  // x-stage workgroup: 16 waves (one per CU), each with an LDS buffer for the FFT exchanges; the
  // tile of 32 rows is written in 256-byte runs (measured 2-4 us faster than 8 waves, 128 bytes).
  // At N = 512 sixteen waves leave 128 registers, which spill 13; eight waves (144 registers, no
  // spill) measured 96 against 128 us at a 512 x 512 scan with 314 pixels.
  static constexpr int kXWaves = N == 512 ? 8 : 16;
  static constexpr int kXStride = kXWaveStride;
  static __device__ __forceinline__ int pad(int i) { return fft_pad(i); }
  static __device__ __forceinline__ void in(int lane, int i, int& b, int& n) { fft_in_index<N>(lane, i, b, n); }
  static __device__ __forceinline__ void out(int lane, int i, int& b, int& m) { fft_out_index<N>(lane, i, b, m); }
  static __device__ __forceinline__ void fill(uint4*, const float2*, int, int) {}
  template <bool EXACT>
  static __device__ __forceinline__ void run(float2* v, float2* buf, const float2* tw, const uint4*, int lane) {
    wave_fft<N>(v, buf, tw, lane);
  }
};

template <int N_, int PREC>
struct XfMfma {
  static constexpr int N = N_;
  static constexpr bool kMfma = true;
  static constexpr int slot_of(int) { return 0; }  // all 16 registers of a lane share its column
  static constexpr int kSlots = 1;
  static constexpr bool kUniformCol = false;        // (the lanes of a wave do not)
  // x-stage workgroup: 16 waves (one workgroup per CU holds the operand tables once); the
  // staging buffer pads one element per 32, so that a lane's outputs (32 apart) hit distinct
  // banks, and the wave stride (8 mod 32 elements) spreads the waves' rows over the banks
  static constexpr int kXWaves = 16;
  static constexpr int kXStride = 1064;
  static __device__ __forceinline__ int pad(int i) { return i + (i >> 5); }
  static __device__ __forceinline__ void in(int lane, int i, int& b, int& n) { MfmaIndex<N>::in(lane, i, b, n); }
  static __device__ __forceinline__ void out(int lane, int i, int& b, int& m) { MfmaIndex<N>::out(lane, i, b, m); }
  static __device__ __forceinline__ void fill(uint4* tab, const float2* tw, int tid, int nthreads) {
    mfma_fill_table<N, PREC>(tab, tw, tid, nthreads);
  }
  template <bool EXACT>
  static __device__ __forceinline__ void run(float2* v, float2*, const float2* tw, const uint4* tab, int lane) {
    mfma_dft<N, PREC, EXACT>(v, tab, tw, lane);
  }
};

template <int N, int PREC>
struct XfSel {
  using type = XfMfma<N, PREC>;
};
template <int N>
struct XfSel<N, STEM_FFT_FP32> {
  using type = XfFft<N>;
};

// f(integral_constant N) for N a power of two in [32, 1024]
template <typename F>
static int with_n(int n, F&& f) {
  switch (n) {
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    default: return STEM_EINVAL;
  }
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// x-stage: rows (kd, ry) with ry in [ry0, ry0 + nr) of D, two real rows per complex transform.
// Tile = 2 W B real rows (B = 1024/N, W waves per workgroup); each wave transforms B row
// pairs; the workgroup then splits the pairs and writes X[kd][m][ry] for m in [0, N/2] in runs
// of consecutive ry.

template <typename XF, typename DT>
__global__ void __launch_bounds__(64 * XF::kXWaves) k_xstage(const DT* __restrict__ D, int ny, int ry0, int nr,
                                                      Magic mnr, int nrows, int pair_store,
                                                      float2* __restrict__ X) {
  constexpr int N = XF::N;
  // counts below 256 are exact in the split formats and need no low part
  constexpr bool kExact = std::is_same<DT, uint8_t>::value;
  __shared__ float2 s_tw[1024];
  constexpr int kThreads = 64 * XF::kXWaves;
  __shared__ float2 s_buf[XF::kXWaves * XF::kXStride];
  __shared__ uint4 s_tab[XF::kMfma ? kMfmaTab : 1];
  constexpr int B = 1024 / N;
  constexpr int TR = 2 * XF::kXWaves * B;  // real rows per tile
  constexpr int NH = N / 2 + 1;
  constexpr int ROWB = N * (int)sizeof(DT);  // bytes per row of D
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  fill_twiddles(s_tw, threadIdx.x, kThreads);
  __syncthreads();
  XF::fill(s_tab, s_tw, threadIdx.x, kThreads);
  if (XF::kMfma) __syncthreads();
  float2* buf = s_buf + wave * XF::kXStride;
  const int ntiles = (nrows + TR - 1) / TR;
  // real row r (< 2^31) -> pixel kd = r / nr and scan row ry0 + r % nr
  auto row_of = [&](int r, int& kd, int& ry) {
    kd = (int)magic_div((uint32_t)r, mnr);
    ry = ry0 + (r - kd * nr);
  };
  // the wave's 2B rows of D as 16-byte chunks, CPL per lane; the next tile's chunks are loaded
  // while this tile is transformed and written
  constexpr int CH = 2 * B * ROWB / 16;
  constexpr int CPL = CH / kWave;
  static_assert(CH % kWave == 0, "row chunks per lane");
  auto load_rows = [&](int tile, uint4* pre) {
    const int r0 = tile * TR + wave * 2 * B;  // first real row of this wave
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int c = lane + kWave * k;
      const int j = c * 16 / ROWB, col = c * 16 % ROWB;
      const int r = r0 + j;
      pre[k] = make_uint4(0u, 0u, 0u, 0u);
      if (r < nrows) {
        int kd, ry;
        row_of(r, kd, ry);
        pre[k] = *(const uint4*)((const char*)D + ((int64_t)kd * ny + ry) * ROWB + col);
      }
    }
  };
  uint4 pre[CPL];
  if ((int)blockIdx.x < ntiles) load_rows(blockIdx.x, pre);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    {
      uint4* raw = (uint4*)buf;
#pragma unroll
      for (int k = 0; k < CPL; ++k) raw[lane + kWave * k] = pre[k];
    }
    if (tile + gridDim.x < ntiles) load_rows(tile + gridDim.x, pre);
    wave_lds_sync();
    float2 v[16];
    {
      const DT* rows = (const DT*)buf;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        XF::in(lane, i, b, n);
        v[i] = make_float2((float)rows[(2 * b) * N + n], (float)rows[(2 * b + 1) * N + n]);
      }
    }
    wave_lds_sync();
    XF::template run<kExact>(v, buf, s_tw, s_tab, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      XF::out(lane, i, b, m);
      buf[XF::pad(b * N + m)] = v[i];
    }
    __syncthreads();
    // split each complex transform z = a + i b of rows (2p, 2p+1) into the two half spectra
    // A(m) = (z(m) + conj z(-m))/2, B(m) = (z(m) - conj z(-m))/(2i); write them at adjacent ry
    for (int u = threadIdx.x; u < NH * (TR / 2); u += kThreads) {
      const int m = u / (TR / 2), pr = u % (TR / 2);
      const int w = pr / B, b = pr % B;
      const float2* wb = s_buf + w * XF::kXStride;
      const float2 z = wb[XF::pad(b * N + m)];
      const float2 zc = cconj(wb[XF::pad(b * N + ((N - m) & (N - 1)))]);
      const float2 va = cscale(cadd(z, zc), 0.5f);
      const float2 vb = cscale(cmul_mi(csub(z, zc)), 0.5f);
      const int rho = tile * TR + 2 * pr;
      int kd, ry;
      row_of(rho, kd, ry);
      if (pair_store && rho + 1 < nrows) {
        *(float4*)(X + ((int64_t)kd * NH + m) * ny + ry) = make_float4(va.x, va.y, vb.x, vb.y);
      } else {
        if (rho < nrows) X[((int64_t)kd * NH + m) * ny + ry] = va;
        if (rho + 1 < nrows) {
          row_of(rho + 1, kd, ry);
          X[((int64_t)kd * NH + m) * ny + ry] = vb;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Fused column transform + Eq. 3.  A wave owns B = 1024/NY consecutive half-spectrum columns c
// (Qx = c*sx) and a group of kept pixels.  For each pixel it loads the row-transformed columns
// X[kd][c][0..NY), transforms them along ry in registers (giving G(kd, (my, c)) for every my),
// and adds every double-overlap term to its accumulators: the direct frequency Q = (my, c) with
// G, and for 0 < c < Nx/2 the mirrored frequency (-my, -c) with conj G.  Only pixels whose set is
// non-empty somewhere in the wave's columns are visited (the active-pixel mask).  The wave writes
// its partial T for its columns into part[g] (column-major [mx][my]); the phase pass sums the
// groups in a fixed order.
//
// Pixels may come in chunks (pixels [k0, k1) of one launch, their columns at X + (kd - xk0) *
// kstride): with `accumulate` a launch adds to the partial sums and counters of the previous
// chunk's launch (same grid, same wave -> partial mapping) instead of overwriting them.
//
// Pruned G: the double-overlap values only, for later sums (refocus) and the adjoint.  For
// scan-frequency column mx in [0, Nx) and pixel kd, the values G(kd, (iy, mx)) for iy in the set of
// that column, ascending iy with the hole [b0, b1] skipped, start at poff[mx * n_k + kd] (column
// major: the runs of a column's pixels follow one another).  Column
// mx <= Nx/2 is half-spectrum column c = mx (direct set); mx > Nx/2 is the mirror of c = Nx - mx,
// whose values are conj G(kd, (-iy, c)).  PWRITE: the fused sum writes them (FINALIZE that keeps
// G); the refocus sum and the adjoint read them (ssb_pruned.h).

// The sets of one pixel for a half-spectrum column c (direct) and for -c (mirror) depend only on
// the geometry; they are tabulated once per reconstruction (k_colsets), 16 bytes per (pixel,
// column): (a0, a1, b0, b1) direct and mirrored as int16 (|iy| <= 2048).
__device__ __forceinline__ void load_colsets(const int4* __restrict__ cst, int64_t i, ColSet& d, ColSet& m) {
  const int4 r = cst[i];
  d = ColSet{(int)(short)(r.x & 0xffff), r.x >> 16, (int)(short)(r.y & 0xffff), r.y >> 16};
  m = ColSet{(int)(short)(r.z & 0xffff), r.z >> 16, (int)(short)(r.w & 0xffff), r.w >> 16};
}

// Arguments shared by the fused column kernels.
struct YArgs {
  const float2* X;          // row-transformed columns, pixel kd at X + (kd - xk0) * kstride
  int xk0;
  const double2* kc;
  const double* kchi;       // chi(Kc) + theta per pixel (general path and adjoint)
  const int4* cst;          // double-overlap interval table [n_k][Nx/2 + 1]
  const uint64_t* cmask;    // active-pixel mask [column set][nmw]
  int nmw, n_k, nx;
  int k0, k1;               // pixels of this launch
  int ngroups;              // pixel groups of [k0, k1)
  int accumulate;           // add to part / wcnt / pdc (a later chunk of pixels)
  const float2* pg;         // pruned G read (refocus, adjoint)
  float2* pgw;              // PWRITE: pruned G written
  const int64_t* poff;      // pruned offsets [Nx][n_k]
  int64_t pcap;             // capacity of the pruned array (entries)
  float2* part;             // partial sums of T [groups][F]
  unsigned long long* wcnt; // per wave: pairs | (8-byte loads << 40)
  const float2* Tbt;        // adjoint: Tbar column-major [mx][my]
  double* pdc;              // adjoint: dL/dc partials [wave][8]
  float* pdth;              // adjoint: dL/dtheta partials [column set][n_k]
  // kernels over the stored values: chi(Kc) + theta evaluated per pixel from kc and theta (may be
  // null) instead of read from kchi
  int kch_inline;
  const float* theta;
  // a call that needs a FINALIZE of the state (refocus, adjoint) passes the state's mark of one and
  // the value a FINALIZE with this layout leaves there; null: no check
  const unsigned long long* ready;
  unsigned long long ready_tag;
  int32_t* status;
};

// A kernel of a call that needs a FINALIZE: true when the state holds none (the first thread of the
// grid reports STEM_ESTATE); the whole workgroup returns then, reading nothing of the state.
__device__ __forceinline__ bool state_unready(const YArgs& a) {
  if (a.ready == nullptr || *a.ready == a.ready_tag) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) report(a.status, STEM_ESTATE);
  return true;
}

constexpr int kLoadShift = 40;  // wcnt packs the pair count below bit 40, the 8-byte loads above

// Position of iy in the compact run of set s ([a0, a1] without the hole [b0, b1]); iy in s.
__device__ __forceinline__ int set_rank(const ColSet& s, int iy) {
  const int h0 = max(s.a0, s.b0), h1 = min(s.a1, s.b1);
  return iy - s.a0 - ((h0 <= h1 && iy > h1) ? h1 - h0 + 1 : 0);
}

__device__ __forceinline__ int set_size(const ColSet& s) {
  if (s.a0 > s.a1) return 0;
  const int h0 = max(s.a0, s.b0), h1 = min(s.a1, s.b1);
  return (s.a1 - s.a0 + 1) - (h0 <= h1 ? h1 - h0 + 1 : 0);
}

// Where the registers of a pixel come from.
struct PixSrc {
  const float2* X;
  int xk0, nx;
  const int4* cst;
  const int64_t* poff;
  const float2* pg;
  int64_t pcap;
};

__device__ __forceinline__ PixSrc pix_src(const YArgs& a) {
  return PixSrc{a.X, a.xk0, a.nx, a.cst, a.poff, a.pg, a.pcap};
}

// Registers of pixel kd for the wave's columns: the row-transformed input in the transform's input
// layout.  Returns the number of 8-byte loads of this lane.
template <typename XF>
__device__ __forceinline__ unsigned load_pixel(const PixSrc a, int kd, int c0, int lane, float2* v) {
  constexpr int NY = XF::N;
  const int nc = a.nx / 2 + 1;
  unsigned n = 0;
  const int64_t kstride = (int64_t)nc * NY;
  const float2* xcol = a.X + (int64_t)(kd - a.xk0) * kstride + (int64_t)c0 * NY;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int b, n_;
    XF::in(lane, i, b, n_);
    const bool in = c0 + b < nc;
    v[i] = in ? xcol[(int64_t)b * NY + n_] : make_float2(0.f, 0.f);
    n += in ? 1u : 0u;
  }
  return n;
}

// the pixels of [kd_a, kd_b) with a non-empty set in column set cs: bits of the active-pixel mask,
// scanned with scalar operations
struct MaskScan {
  const uint64_t* mrow;
  int kd_b;
  int mw = -1;
  uint64_t mword = 0;
  __device__ __forceinline__ int next(int from) {
    for (int kd = from; kd < kd_b;) {
      const int w = kd >> 6;
      if (w != mw) {
        mw = w;
        mword = mrow[w];
      }
      const uint64_t bits = mword >> (kd & 63);
      if (bits) {
        kd += __builtin_ctzll(bits);
        return kd < kd_b ? kd : kd_b;
      }
      kd = (w + 1) << 6;
    }
    return kd_b;
  }
};

// CHI0: the aberration function and theta are identically zero, so every phase factor of Eq. 3
// is exactly 1 and the sum adds G itself (conj G for mirrored frequencies): the same values the
// general path produces for chi = 0, without evaluating them.

template <typename XF, bool CHI0, bool PWRITE>
__global__ void __launch_bounds__(kYThreads, 2) k_yreduce(YArgs a, Optics o) {
  if (state_unready(a)) return;
  constexpr int NY = XF::N;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[XF::kMfma ? 1 : 4 * kXWaveStride];
  __shared__ uint4 s_tab[XF::kMfma ? kMfmaTab : 1];
  constexpr int B = 1024 / NY;
  using SL = XF;
  constexpr int kSlotStride = 16 / SL::kSlots;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = a.nx;
  const int nc = nx / 2 + 1;
  const int ncs = (nc + B - 1) / B;                       // column sets
  const int g = blockIdx.x % a.ngroups;
  const int cs = (blockIdx.x / a.ngroups) * 4 + wave;     // this wave's column set
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  const PixSrc src = pix_src(a);
  fill_twiddles(s_tw, threadIdx.x, kYThreads);
  __syncthreads();
  XF::fill(s_tab, s_tw, threadIdx.x, kYThreads);
  if (XF::kMfma) __syncthreads();
  if (cs >= ncs) {
    if (lane == 0 && !a.accumulate) a.wcnt[wid] = 0ull;
    return;
  }
  float2* buf = s_buf + wave * kXWaveStride;
  const int c0 = cs * B;
  const int kd_a = a.k0 + (int)((int64_t)(a.k1 - a.k0) * g / a.ngroups);
  const int kd_b = a.k0 + (int)((int64_t)(a.k1 - a.k0) * (g + 1) / a.ngroups);
  float2 accd[16], accm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) accd[i] = accm[i] = make_float2(0.f, 0.f);
  unsigned cnt = 0, nld = 0;
  MaskScan ms{a.cmask + (int64_t)cs * a.nmw, kd_b};
  // the columns of the next active pixel (of the next two on the zero-aberration path, whose sum
  // leaves the registers for it) are loaded while this one is transformed and summed; at N = 512
  // the second pixel's columns spill (12 registers) and one ahead is faster (75 against 97 us at
  // a 512 x 512 scan with 314 pixels)
  constexpr int kAhead =
      (CHI0 && !PWRITE && ((!XF::kMfma && XF::kUniformCol && NY != 512) || (XF::kMfma && NY == 1024))) ? 2 : 1;
  int kd = ms.next(kd_a);
  int kd1 = kAhead == 2 && kd < kd_b ? ms.next(kd + 1) : kd_b;
  float2 v[16], v1[kAhead == 2 ? 16 : 1];
  if (kd < kd_b) nld += load_pixel<XF>(src, kd, c0, lane, v);
  if constexpr (kAhead == 2) {
    if (kd1 < kd_b) nld += load_pixel<XF>(src, kd1, c0, lane, v1);
  }
  while (kd < kd_b) {
    int kdn;
    float2 vn[16];
    if constexpr (kAhead == 2) {
      kdn = kd1;
      kd1 = kd1 < kd_b ? ms.next(kd1 + 1) : kd_b;
      if (kd1 < kd_b) nld += load_pixel<XF>(src, kd1, c0, lane, vn);
    } else {
      kdn = ms.next(kd + 1);
      if (kdn < kd_b) nld += load_pixel<XF>(src, kdn, c0, lane, vn);
    }
    const double2 k = a.kc[kd];
    // double-overlap sets of this pixel for the lane's columns (direct and mirrored)
    ColSet sd[SL::kSlots], sm[SL::kSlots];
#pragma unroll
    for (int sl = 0; sl < SL::kSlots; ++sl) {
      int b0, m0;
      XF::out(lane, sl * kSlotStride, b0, m0);
      const int c = c0 + b0;
      sd[sl] = ColSet{1, 0, 1, 0};
      sm[sl] = ColSet{1, 0, 1, 0};
      if (c < nc) load_colsets(a.cst, (int64_t)kd * nc + c, sd[sl], sm[sl]);
    }
    XF::template run<false>(v, buf, s_tw, s_tab, lane);
    if constexpr (PWRITE) {
      // the double-overlap values of this pixel into the pruned array
#pragma unroll
      for (int sl = 0; sl < SL::kSlots; ++sl) {
        int b0, m0;
        XF::out(lane, sl * kSlotStride, b0, m0);
        const int c = c0 + b0;
        int64_t pd = 0, pm = 0;
        if (c < nc) {
          pd = a.poff[(int64_t)c * a.n_k + kd];
          if (c > 0 && 2 * c < nx) pm = a.poff[(int64_t)(nx - c) * a.n_k + kd];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          if (SL::slot_of(i) != sl) continue;
          int b, m;
          XF::out(lane, i, b, m);
          const int iy = signed_index(m, NY), jy = signed_index((NY - m) & (NY - 1), NY);
          if (c < nc && sd[sl].has(iy)) {
            const int64_t e = pd + set_rank(sd[sl], iy);
            if (e >= 0 && e < a.pcap) a.pgw[e] = v[i];
          }
          if (c < nc && sm[sl].has(jy)) {
            const int64_t e = pm + set_rank(sm[sl], jy);
            if (e >= 0 && e < a.pcap) a.pgw[e] = cconj(v[i]);
          }
        }
      }
    }
    if constexpr (CHI0 && !XF::kMfma && XF::kUniformCol) {
      // Every register of a slot belongs to one column; the lane's frequencies in it are
      // m = lane + 64 j, j = 0 .. N/64 - 1.  In signed order iy = 64 p - (N/2 - lane) with
      // p = (j + N/128) mod N/64, so each interval of a double-overlap set is a run of p, formed
      // once per pixel as a bit mask; a register then adds its value times its bit (1 adds the
      // value exactly, 0 adds nothing).
      constexpr int NP = NY / 64;
      static_assert(NP == (XF::NB / 64) * XF::RL, "register layout of the uniform-column transform");
      const int base = NY / 2 - lane;
      auto pbits = [&](int lo, int hi) -> uint32_t {  // p with lo <= iy(p) <= hi
        int p0 = (lo + base + 63) >> 6, p1 = (hi + base) >> 6;
        p0 = p0 < 0 ? 0 : p0;
        p1 = p1 > NP - 1 ? NP - 1 : p1;
        return p1 >= p0 ? (2u << p1) - (1u << p0) : 0u;
      };
      uint32_t md[SL::kSlots], mm[SL::kSlots];
#pragma unroll
      for (int sl = 0; sl < SL::kSlots; ++sl) {
        md[sl] = pbits(sd[sl].a0, sd[sl].a1) & ~pbits(sd[sl].b0, sd[sl].b1);
        // mirrored frequency jy = -iy, except iy = -N/2 (lane 0, p = 0), which is its own mirror
        mm[sl] = pbits(-sm[sl].a1, -sm[sl].a0) & ~pbits(-sm[sl].b1, -sm[sl].b0);
        if (lane == 0) mm[sl] = (mm[sl] & ~1u) | (sm[sl].has(-NY / 2) ? 1u : 0u);
        cnt += __builtin_popcount(md[sl]) + __builtin_popcount(mm[sl]);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int sl = SL::slot_of(i);
        const int j = (i / XF::RL) % (XF::NB / 64) + (XF::NB / 64) * (i % XF::RL);
        const int pb = (j + NP / 2) % NP;
        const float wd = (float)((md[sl] >> pb) & 1u), wm = (float)((mm[sl] >> pb) & 1u);
        accd[i].x = fmaf(v[i].x, wd, accd[i].x);
        accd[i].y = fmaf(v[i].y, wd, accd[i].y);
        accm[i].x = fmaf(v[i].x, wm, accm[i].x);
        accm[i].y = fmaf(-v[i].y, wm, accm[i].y);
      }
    } else if constexpr (CHI0 && XF::kMfma && NY >= 64) {
      // Matrix-core layout: the lane's 16 frequencies are m = 32 (c mod N/32) + q, c = lane mod 32,
      // with q = 8 (i/4) + 4 h + i mod 4, h = lane / 32: one aligned block of 32 that never
      // straddles N/2, so in signed order iy = base + q and each interval of a double-overlap set
      // is a run of q, formed once per pixel as a bit mask (as in the uniform-column sum above).
      static_assert(SL::kSlots == 1, "one column per lane in the matrix-core layout");
      const int h = lane >> 5;
      const int mb = 32 * ((lane & 31) % (NY / 32));
      const int base = mb < NY / 2 ? mb : mb - NY;
      auto qbits = [&](int lo, int hi) -> uint32_t {  // q in [0, 32) with lo <= base + q <= hi
        int q0 = lo - base, q1 = hi - base;
        q0 = q0 < 0 ? 0 : q0;
        q1 = q1 > 31 ? 31 : q1;
        return q1 >= q0 ? (2u << q1) - (1u << q0) : 0u;  // 2u << 31 wraps to 0: bits q0..31
      };
      uint32_t md = qbits(sd[0].a0, sd[0].a1) & ~qbits(sd[0].b0, sd[0].b1);
      uint32_t mm = qbits(-sm[0].a1, -sm[0].a0) & ~qbits(-sm[0].b1, -sm[0].b0);
      // iy = -N/2 (the block's q = 0 when base = -N/2) is its own mirror
      if (base == -NY / 2) mm = (mm & ~1u) | (sm[0].has(-NY / 2) ? 1u : 0u);
      const uint32_t own = 0x0f0f0f0fu << (4 * h);  // the q of this lane's registers
      cnt += __builtin_popcount(md & own) + __builtin_popcount(mm & own);
      md >>= 4 * h;
      mm >>= 4 * h;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int q = 8 * (i >> 2) + (i & 3);
        uint32_t bd = (md >> q) & 1u, bm = (mm >> q) & 1u;
        // one register's weights at a time: formed all at once, the 32 weights cost registers
        asm volatile("" : "+v"(bd), "+v"(bm));
        const float wd = (float)bd, wm = (float)bm;
        accd[i].x = fmaf(v[i].x, wd, accd[i].x);
        accd[i].y = fmaf(v[i].y, wd, accd[i].y);
        accm[i].x = fmaf(v[i].x, wm, accm[i].x);
        accm[i].y = fmaf(-v[i].y, wm, accm[i].y);
      }
    } else if constexpr (CHI0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int sl = SL::slot_of(i);
        int b, m;
        XF::out(lane, i, b, m);
        asm volatile("" : "+v"(m));
        if (sd[sl].has(signed_index(m, NY))) {
          accd[i].x += v[i].x;
          accd[i].y += v[i].y;
          ++cnt;
        }
        if (sm[sl].has(signed_index((NY - m) & (NY - 1), NY))) {
          accm[i].x += v[i].x;
          accm[i].y -= v[i].y;
          ++cnt;
        }
      }
    } else {
      if constexpr (SL::kSlots > 1) {
        const double kch = a.kchi[kd];
#pragma unroll
        for (int sl = 0; sl < SL::kSlots; ++sl) {
          int b0, m0;
          XF::out(lane, sl * kSlotStride, b0, m0);
          // one column polynomial live at a time: the slot's direct frequencies, then its mirrored
          // ones, each polynomial formed only after the previous pass (formed all at once they stay
          // live together and spill at N = 512, two slots per lane)
          asm volatile("" : "+v"(b0));
          const int c = c0 + b0;
          {
            const ChiCol chd = chi_column(o.lk * (k.x - (double)signed_index(c, nx) * o.sx), o);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              if (SL::slot_of(i) != sl) continue;
              int b, m;
              XF::out(lane, i, b, m);
              // keep the per-register frequency arithmetic inside the pixel loop: hoisted out of it,
              // the 16 registers' frequencies stay live across the loop and cost occupancy
              asm volatile("" : "+v"(m));
              const int iy = signed_index(m, NY);
              if (sd[sl].has(iy)) {
                const double wy = o.lk * (k.y - (double)iy * o.sy);
                const float2 e = expi_reduced(chi_eval(chd, wy) - kch);
                accd[i].x += v[i].x * e.x - v[i].y * e.y;
                accd[i].y += v[i].x * e.y + v[i].y * e.x;
                ++cnt;
              }
            }
          }
          int cm = c;
          asm volatile("" : "+v"(cm));
          {
            const ChiCol chm = chi_column(o.lk * (k.x - (double)signed_index(nx - cm, nx) * o.sx), o);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              if (SL::slot_of(i) != sl) continue;
              int b, m;
              XF::out(lane, i, b, m);
              asm volatile("" : "+v"(m));
              const int jy = signed_index((NY - m) & (NY - 1), NY);
              if (sm[sl].has(jy)) {
                const double wy = o.lk * (k.y - (double)jy * o.sy);
                const float2 e = expi_reduced(chi_eval(chm, wy) - kch);
                accm[i].x += v[i].x * e.x + v[i].y * e.y;
                accm[i].y += v[i].x * e.y - v[i].y * e.x;
                ++cnt;
              }
            }
          }
        }
      } else {
        const double kch = a.kchi[kd];
#pragma unroll
        for (int sl = 0; sl < SL::kSlots; ++sl) {
          int b0, m0;
          XF::out(lane, sl * kSlotStride, b0, m0);
          const int c = c0 + b0;
          const ChiCol chd = chi_column(o.lk * (k.x - (double)signed_index(c, nx) * o.sx), o);
          const ChiCol chm = chi_column(o.lk * (k.x - (double)signed_index(nx - c, nx) * o.sx), o);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (SL::slot_of(i) != sl) continue;
            int b, m;
            XF::out(lane, i, b, m);
            // keep the per-register frequency arithmetic inside the pixel loop: hoisted out of it, the
            // 16 registers' frequencies stay live across the loop and cost occupancy
            asm volatile("" : "+v"(m));
            const int iy = signed_index(m, NY);
            if (sd[sl].has(iy)) {
              const double wy = o.lk * (k.y - (double)iy * o.sy);
              const float2 e = expi_reduced(chi_eval(chd, wy) - kch);
              accd[i].x += v[i].x * e.x - v[i].y * e.y;
              accd[i].y += v[i].x * e.y + v[i].y * e.x;
              ++cnt;
            }
            const int jy = signed_index((NY - m) & (NY - 1), NY);
            if (sm[sl].has(jy)) {
              const double wy = o.lk * (k.y - (double)jy * o.sy);
              const float2 e = expi_reduced(chi_eval(chm, wy) - kch);
              accm[i].x += v[i].x * e.x + v[i].y * e.y;
              accm[i].y += v[i].x * e.y - v[i].y * e.x;
              ++cnt;
            }
          }
        }
      }
    }
    kd = kdn;
    if constexpr (kAhead == 2) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        v[i] = v1[i];
        v1[i] = vn[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = vn[i];
    }
  }
  float2* pgp = a.part + (int64_t)g * nx * NY;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int b, m;
    XF::out(lane, i, b, m);
    const int c = c0 + b;
    if (c >= nc) continue;
    float2* pd = pgp + (int64_t)c * NY + m;
    float2* pm = pgp + (int64_t)(nx - c) * NY + ((NY - m) & (NY - 1));
    const bool mir = c > 0 && 2 * c < nx;
    if (a.accumulate) {
      *pd = cadd(*pd, accd[i]);
      if (mir) *pm = cadd(*pm, accm[i]);
    } else {
      *pd = accd[i];
      if (mir) *pm = accm[i];
    }
  }
  unsigned long long cc = (unsigned long long)cnt + ((unsigned long long)nld << kLoadShift);
  for (int off = 32; off > 0; off >>= 1) cc += __shfl_xor(cc, off);
  if (lane == 0) a.wcnt[wid] = a.accumulate ? a.wcnt[wid] + cc : cc;
}

template <typename XF>
constexpr bool slots_consecutive() {
  for (int i = 0; i < 16; ++i)
    if (XF::slot_of(i) != i / (16 / XF::kSlots)) return false;
  return true;
}

// Fused column transform + adjoint of Eq. 3.  Same work split as k_yreduce (also over chunks of
// pixels, with `accumulate`).  For every double-overlap pair, z = G e^{i psi} (conj G for mirrored
// frequencies), w = Re(conj(Tbar(Q)) i z); dL/dc_j gains w (B_j(K - Q) - B_j(K)) and
// dL/dtheta[kd] loses w.  Along one column (fixed wx = lam dk (Kx - Qx)) every B_j(K - Q) is a
// polynomial of degree <= 4 in wy = lam dk (Ky - Qy) whose coefficients are polynomials in wx, so
// the pairs of a (pixel, column) are reduced to the moments M_n = sum w wy^n, n = 0..4, and the
// eight gradient terms follow from them once per (pixel, column); sum w B_j(K) is B_j(K) times the
// pixel's sum of w.  Partials: pdc[wave][8] (FP64), pdth[column set][kd] (FP32; one writer).
template <typename XF>
__global__ void __launch_bounds__(kYThreads, 2) k_yadjoint(YArgs a, Optics o) {
  if (state_unready(a)) return;
  static_assert(slots_consecutive<XF>(), "the registers of a slot are consecutive");
  constexpr int NY = XF::N;
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[XF::kMfma ? 1 : 4 * kXWaveStride];
  __shared__ uint4 s_tab[XF::kMfma ? kMfmaTab : 1];
  constexpr int B = 1024 / NY;
  constexpr int kSlotStride = 16 / XF::kSlots;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = a.nx;
  const int nc = nx / 2 + 1;
  const int ncs = (nc + B - 1) / B;
  const int g = blockIdx.x % a.ngroups;
  const int cs = (blockIdx.x / a.ngroups) * 4 + wave;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  const PixSrc src = pix_src(a);
  fill_twiddles(s_tw, threadIdx.x, kYThreads);
  __syncthreads();
  XF::fill(s_tab, s_tw, threadIdx.x, kYThreads);
  if (XF::kMfma) __syncthreads();
  if (cs >= ncs) {
    if (lane < 8 && !a.accumulate) a.pdc[wid * 8 + lane] = 0.0;
    return;
  }
  float2* buf = s_buf + wave * kXWaveStride;
  const int c0 = cs * B;
  const int kd_a = a.k0 + (int)((int64_t)(a.k1 - a.k0) * g / a.ngroups);
  const int kd_b = a.k0 + (int)((int64_t)(a.k1 - a.k0) * (g + 1) / a.ngroups);
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  const double s2pi = 6.283185307179586476925286766559 / o.lam;
  float* pth = a.pdth + (int64_t)cs * a.n_k;
  MaskScan ms{a.cmask + (int64_t)cs * a.nmw, kd_b};
  int done = kd_a;  // pixels below `done` have their dL/dtheta partial written
  int kd = ms.next(kd_a);
  float2 v[16];
  if (kd < kd_b) load_pixel<XF>(src, kd, c0, lane, v);
  while (kd < kd_b) {
    const int kdn = ms.next(kd + 1);
    float2 vn[16];
    if (kdn < kd_b) load_pixel<XF>(src, kdn, c0, lane, vn);
    if (lane == 0)
      for (int z = done; z < kd; ++z) pth[z] = 0.f;  // pixels without pairs in these columns
    const double2 k = a.kc[kd];
    ColSet sd[XF::kSlots], sm[XF::kSlots];
#pragma unroll
    for (int sl = 0; sl < XF::kSlots; ++sl) {
      int b0, m0;
      XF::out(lane, sl * kSlotStride, b0, m0);
      const int c = c0 + b0;
      sd[sl] = ColSet{1, 0, 1, 0};
      sm[sl] = ColSet{1, 0, 1, 0};
      if (c < nc) load_colsets(a.cst, (int64_t)kd * nc + c, sd[sl], sm[sl]);
    }
    XF::template run<false>(v, buf, s_tw, s_tab, lane);
    const double kch = a.kchi[kd];
    double wl = 0.0;  // this lane's sum of w over the pixel's pairs
#pragma unroll
    for (int sl = 0; sl < XF::kSlots; ++sl) {
      int b0, m0;
      XF::out(lane, sl * kSlotStride, b0, m0);
      const int c = c0 + b0;
      for (int side = 0; side < 2; ++side) {
        const int ix = signed_index(side ? nx - c : c, nx);
        const double wx = o.lk * (k.x - (double)ix * o.sx);
        const ChiCol ch = chi_column(wx, o);
        double M0 = 0.0, M1 = 0.0, M2 = 0.0, M3 = 0.0, M4 = 0.0;
        bool any = false;
        // the pairs of register i: w = Re(conj(Tbar) i z) into the moments
        auto pair = [&](int i, int m, int iy, float2 tb) {
          const double wy = o.lk * (k.y - (double)iy * o.sy);
          const float2 e = expi_reduced(chi_eval(ch, wy) - kch);
          const float2 gq = side ? cconj(v[i]) : v[i];
          const float2 z = make_float2(gq.x * e.x - gq.y * e.y, gq.x * e.y + gq.y * e.x);
          const double w = (double)(tb.x * (-z.y) + tb.y * z.x);
          any = true;
          double t = w;
          M0 += t;
          t *= wy;
          M1 += t;
          t *= wy;
          M2 += t;
          t *= wy;
          M3 += t;
          t *= wy;
          M4 += t;
          (void)m;
        };
        if constexpr (XF::kSlots == 1) {
          // Tbar at the pairs' frequencies: first the loads of every register holding a pair in some
          // lane of the wave (one uniform branch each, so that they issue together), then the
          // pairs; kept in registers for every frequency of the lane across the pixel loop, Tbar
          // would cost occupancy
          float2 tbv[16];
          uint32_t hasp = 0;  // registers with a pair in this lane
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            int b, m;
            XF::out(lane, i, b, m);
            const int iy = side ? signed_index((NY - m) & (NY - 1), NY) : signed_index(m, NY);
            const bool ok = c < nc && (side ? sm[sl].has(iy) : sd[sl].has(iy));  // mirror empty unless 0 < c < Nx/2
            hasp |= ok ? 1u << i : 0u;
            tbv[i] = make_float2(0.f, 0.f);
            if (__ballot(ok)) {
              const int cq = c < nc ? c : nc - 1;
              const int col = side ? (nx - cq) % nx : cq;
              tbv[i] = a.Tbt[(int64_t)col * NY + (side ? ((NY - m) & (NY - 1)) : m)];
            }
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (!((hasp >> i) & 1u)) continue;
            int b, m;
            XF::out(lane, i, b, m);
            asm volatile("" : "+v"(m));  // see k_yreduce
            pair(i, m, side ? signed_index((NY - m) & (NY - 1), NY) : signed_index(m, NY), tbv[i]);
          }
        } else {
          // several columns per wave: each lane reads Tbar at its register's frequency (a clamped
          // address past the half spectrum), then the pair
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (XF::slot_of(i) != sl) continue;
            int b, m;
            XF::out(lane, i, b, m);
            asm volatile("" : "+v"(m));  // see k_yreduce
            const int iy = side ? signed_index((NY - m) & (NY - 1), NY) : signed_index(m, NY);
            const int cq = c < nc ? c : nc - 1;
            const int col = side ? (nx - cq) % nx : cq;
            const float2 tb = a.Tbt[(int64_t)col * NY + (side ? ((NY - m) & (NY - 1)) : m)];
            if (c >= nc || !(side ? sm[sl].has(iy) : sd[sl].has(iy))) continue;  // mirror empty unless 0 < c < Nx/2
            pair(i, m, iy, tb);
          }
        }
        if (any) {
          // sum over the column's pairs of w B_j(K - Q), B_j as polynomials in wy
          const double x2 = wx * wx, x3 = x2 * wx, x4 = x2 * x2;
          dc[0] += 0.5 * s2pi * (x2 * M0 + M2);
          dc[1] += 0.5 * s2pi * (x2 * M0 - M2);
          dc[2] += s2pi * (wx * M1);
          dc[3] += (s2pi / 3.0) * (x3 * M0 + wx * M2);
          dc[4] += (s2pi / 3.0) * (x2 * M1 + M3);
          dc[5] += (s2pi / 3.0) * (x3 * M0 - 3.0 * wx * M2);
          dc[6] += (s2pi / 3.0) * (3.0 * x2 * M1 - M3);
          dc[7] += 0.25 * s2pi * (x4 * M0 + 2.0 * x2 * M2 + M4);
          wl += M0;
        }
      }
    }
    if (wl != 0.0) {
      double bk[8];
      chi_basis(k.x, k.y, o, bk);
#pragma unroll
      for (int j = 0; j < 8; ++j) dc[j] -= bk[j] * wl;
    }
    float wsum = (float)wl;
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
    if (lane == 0) pth[kd] = -wsum;
    done = kd + 1;
    kd = kdn;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = vn[i];
  }
  if (lane == 0)
    for (int z = done; z < kd_b; ++z) pth[z] = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double t = dc[j];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) a.pdc[wid * 8 + j] = a.accumulate ? a.pdc[wid * 8 + j] + t : t;
  }
}

// ---------------------------------------------------------------------------------------------
// launchers, one instantiation per precision

template <int PREC, typename DT>
int launch_xstage_p(int nx, const DT* D, int ny, int ry0, int nr, int64_t nrows, float2* X, hipStream_t s) {
  // rows 2p, 2p+1 of a tile share a pixel and sit at adjacent, 16-byte aligned ry when the
  // chunk starts on an even row and holds an even number of rows per pixel
  const int pair_store = (nr % 2 == 0) && (ry0 % 2 == 0);
  // rows are counted in 32 bits (n_K * Ny is far below 2^31 for any cube that fits in memory)
  if (nrows <= 0 || nrows > ((int64_t)1 << 31) - 4096 || nr <= 0) return nrows == 0 ? STEM_OK : STEM_EINVAL;
  STEM_TRACE(PREC == STEM_FFT_FP32 ? "xstage_fft" : "xstage_mfma", s);
  const int st = with_n(nx, [&](auto nc) {
    using XF = typename XfSel<decltype(nc)::value, PREC>::type;
    const int64_t tr = 2 * XF::kXWaves * (1024 / nx);
    const int64_t tiles = (nrows + tr - 1) / tr;
    // every workgroup resident, each streaming its tiles with the next tile's rows in flight
    const int res = resident_blocks((const void*)k_xstage<XF, DT>, 64 * XF::kXWaves);
    const int64_t cap = res > 0 ? res : 4096;
    const dim3 grid((unsigned)(tiles < cap ? tiles : cap)), blk(64 * XF::kXWaves);
    hipLaunchKernelGGL((k_xstage<XF, DT>), grid, blk, 0, s, D, ny, ry0, nr, make_magic((uint32_t)nr), (int)nrows,
                       pair_store, X);
  });
  if (st) return st;
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// grid of the fused column kernels: column sets in fours (one per wave) times pixel groups
inline dim3 ygrid(int ny, int nx, int ngroups) {
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  return dim3((unsigned)(((ncs + 3) / 4) * ngroups));
}

// the fused sum over pixels [a.k0, a.k1) with the transform policy of precision PREC; pwrite: also
// write the pruned G
template <int PREC>
int launch_yreduce_p(int ny, const YArgs& a, const Optics& o, int chi0, int pwrite, hipStream_t s) {
  const dim3 grid = ygrid(ny, a.nx, a.ngroups), blk(kYThreads);
  STEM_TRACE(PREC == STEM_FFT_FP32 ? "ssb_yreduce" : "ssb_yreduce_mfma", s);
  const int st = with_n(ny, [&](auto nc) {
    using XF = typename XfSel<decltype(nc)::value, PREC>::type;
    if (chi0 && pwrite)
      hipLaunchKernelGGL((k_yreduce<XF, true, true>), grid, blk, 0, s, a, o);
    else if (chi0)
      hipLaunchKernelGGL((k_yreduce<XF, true, false>), grid, blk, 0, s, a, o);
    else if (pwrite)
      hipLaunchKernelGGL((k_yreduce<XF, false, true>), grid, blk, 0, s, a, o);
    else
      hipLaunchKernelGGL((k_yreduce<XF, false, false>), grid, blk, 0, s, a, o);
  });
  if (st) return st;
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

template <int PREC>
int launch_yadjoint_p(int ny, const YArgs& a, const Optics& o, hipStream_t s) {
  const dim3 grid = ygrid(ny, a.nx, a.ngroups), blk(kYThreads);
  STEM_TRACE(PREC == STEM_FFT_FP32 ? "ssb_yadjoint" : "ssb_yadjoint_mfma", s);
  const int st = with_n(ny, [&](auto nc) {
    using XF = typename XfSel<decltype(nc)::value, PREC>::type;
    hipLaunchKernelGGL((k_yadjoint<XF>), grid, blk, 0, s, a, o);
  });
  if (st) return st;
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

extern template int launch_xstage_p<STEM_DFT_BF16_SPLIT, uint8_t>(int, const uint8_t*, int, int, int, int64_t, float2*, hipStream_t);
extern template int launch_xstage_p<STEM_DFT_BF16_SPLIT, uint16_t>(int, const uint16_t*, int, int, int, int64_t, float2*, hipStream_t);
extern template int launch_yreduce_p<STEM_DFT_BF16_SPLIT>(int, const YArgs&, const Optics&, int, int, hipStream_t);
extern template int launch_yadjoint_p<STEM_DFT_BF16_SPLIT>(int, const YArgs&, const Optics&, hipStream_t);
extern template int launch_xstage_p<STEM_DFT_FP16_SPLIT, uint8_t>(int, const uint8_t*, int, int, int, int64_t, float2*, hipStream_t);
extern template int launch_xstage_p<STEM_DFT_FP16_SPLIT, uint16_t>(int, const uint16_t*, int, int, int, int64_t, float2*, hipStream_t);
extern template int launch_yreduce_p<STEM_DFT_FP16_SPLIT>(int, const YArgs&, const Optics&, int, int, hipStream_t);
extern template int launch_yadjoint_p<STEM_DFT_FP16_SPLIT>(int, const YArgs&, const Optics&, hipStream_t);

}  // namespace stem
