// Single-sideband (SSB) ptychography from linear-index events (Sec. IV) and its adjoint.
//
// Pipeline (state buffer owned by the caller):
//   k_geometry     kept binned pixels (rows of the bright-field disk) and their centres Kc
//   k_bin          events -> D[kd][ry][rx] (uint8/uint16 counts)                    (Table 1)
//   k_xstage       real row FFT along rx, output transposed X[kd][mx][ry], mx in [0, Nx/2]
//   y-stage        FFT along ry of every (kd, mx) column, in place: G[kd][mx][my]   (Eq. 2)
//   k_reduce       Eq. 3 over the double-overlap set for every Q -> T[mx][my]
//   phase          two inverse row FFT passes -> phi = Im IFFT2(T)
// The other half of the Q plane (mx > Nx/2) uses G(K, Q) = conj G(K, -Q) of the real input.
#include "common.h"
#include "fft_wave.h"
#include "ssb_fused.h"
#include "kernels.h"
#include "optics.h"
#include "trace.h"

namespace stem {

constexpr int kMaxPixels = 4096;

struct SsbLayout {
  int n_k, nby, nh;
  int64_t F;
  size_t rows, kc, kchi, cst, cmask, lut, stats, D, X, T, A, Tb, pdc, pdth, part, wcnt, total;
  int nmw;      // 64-bit words per column set of the active-pixel mask
  int groups;  // pixel groups of the fused column transform + sum
  int ncs;     // column sets (B = 1024/Ny half-spectrum columns each)
  int64_t nwy; // waves of the fused kernels
  int64_t nblk;  // workgroups of the per-Q kernels
};

static int yreduce_groups(int ny, int nx, int n_k);

static int count_pixels(const stem_det& det, double r2) {
  const int nbx = det.W / det.bin, nby = det.H / det.bin;
  int n = 0;
  for (int by = 0; by < nby; ++by) {
    int lo, hi;
    kept_run(det.bin, by, nbx, det.cx, det.cy, r2, lo, hi);
    n += hi - lo;
  }
  return n;
}

static bool det_ok(const stem_det* d) {
  return d && d->W > 0 && d->H > 0 && (int64_t)d->W * d->H < (1ll << 31) && d->bin >= 1 &&
         d->W % d->bin == 0 && d->H % d->bin == 0 && d->H / d->bin <= 4096;
}

static bool optics_ok(const stem_optics* o) {
  if (!o || !(o->r_bf > 0) || !(o->dk > 0) || !(o->lam > 0)) return false;
  for (int j = 0; j < 8; ++j)
    if (!(o->c[j] == o->c[j]) || o->c[j] > 1e300 || o->c[j] < -1e300) return false;
  return true;
}

static size_t make_layout(const stem_det& det, const stem_scan& scan, const stem_ssb& ssb, int n_k,
                          SsbLayout* L) {
  L->n_k = n_k;
  L->nby = det.H / det.bin;
  L->nh = scan.nx / 2 + 1;
  L->F = (int64_t)scan.ny * scan.nx;
  L->nblk = (L->F + 255) / 256;
  size_t o = 0;
  L->rows = o;  o = align256(o + sizeof(RowRun) * L->nby);
  L->kc = o;    o = align256(o + sizeof(double2) * n_k);
  L->kchi = o;  o = align256(o + sizeof(double) * n_k);
  L->cst = o;   o = align256(o + sizeof(int4) * n_k * L->nh);
  L->nmw = (n_k + 63) / 64;
  L->cmask = o; o = align256(o + sizeof(uint64_t) * (size_t)L->nmw * ((L->nh + 1024 / scan.ny - 1) / (1024 / scan.ny)));
  L->lut = o;   o = align256(o + sizeof(int16_t) * (size_t)det.W * det.H);
  L->stats = o; o = align256(o + sizeof(unsigned long long) * 4);
  L->D = o;     o = align256(o + (size_t)n_k * L->F * (ssb.d_bits / 8));
  L->X = o;     o = align256(o + (size_t)n_k * L->nh * scan.ny * sizeof(float2));
  L->T = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->A = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->Tb = o;    o = align256(o + (size_t)L->F * sizeof(float2));
  L->groups = yreduce_groups(scan.ny, scan.nx, n_k);
  {
    const int B = 1024 / scan.ny;
    L->ncs = (L->nh + B - 1) / B;                          // column sets of the fused kernels
    L->nwy = (int64_t)((L->ncs + 3) / 4) * 4 * L->groups;  // their waves
  }
  L->pdc = o;   o = align256(o + (size_t)L->nwy * 8 * sizeof(double));
  L->pdth = o;  o = align256(o + (size_t)L->ncs * n_k * sizeof(float));
  L->part = o;  o = align256(o + (size_t)L->groups * L->F * sizeof(float2));
  L->wcnt = o;  o = align256(o + (size_t)L->nwy * sizeof(unsigned long long));
  L->total = o;
  return o;
}

// ---------------------------------------------------------------------------------------------
// precision dispatch of the scan-DFT launchers

template <typename DT>
static int launch_xstage_t(int prec, int nx, const DT* D, int ny, int ry0, int nr, int64_t nrows, float2* X,
                           hipStream_t s) {
  switch (prec) {
    case STEM_DFT_BF16_SPLIT: return launch_xstage_p<STEM_DFT_BF16_SPLIT, DT>(nx, D, ny, ry0, nr, nrows, X, s);
    case STEM_DFT_FP16_SPLIT: return launch_xstage_p<STEM_DFT_FP16_SPLIT, DT>(nx, D, ny, ry0, nr, nrows, X, s);
    default: return launch_xstage_p<STEM_FFT_FP32, DT>(nx, D, ny, ry0, nr, nrows, X, s);
  }
}

// Double-overlap intervals of every (pixel, half-spectrum column) and of its mirror, and the
// active-pixel mask: bit j of word (cs, w) is set when pixel 64 w + j has a non-empty set in some
// column of column set cs (B = 1024/Ny consecutive half-spectrum columns).  One wave per mask
// word: lane j takes pixel 64 w + j over the columns of the set, a ballot packs the 64 answers.
// Workgroups past the mask's also tabulate chi(Kc) + theta per pixel and reset the counters of
// the sum that follows (the work of k_chi_table), when kchi is given.
__global__ void __launch_bounds__(256) k_colsets(const double2* __restrict__ kc, int n_k, int nx, int ny, Optics o,
                                                 int B, int ncs, int nmw, int4* __restrict__ cst,
                                                 uint64_t* __restrict__ mask, int mask_blocks,
                                                 const float* __restrict__ theta, double* __restrict__ kchi,
                                                 unsigned long long* __restrict__ stats, int groups) {
  if ((int)blockIdx.x >= mask_blocks) {
    const int kd = (blockIdx.x - mask_blocks) * blockDim.x + threadIdx.x;
    if (kd < 4) stats[kd] = kd == 1 ? (unsigned long long)groups : 0ull;
    if (kd < n_k) {
      const double2 k = kc[kd];
      kchi[kd] = chi_poly(k.x, k.y, o) + (theta ? (double)theta[kd] : 0.0);
    }
    return;
  }
  const int64_t word = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (word >= (int64_t)ncs * nmw) return;  // uniform across the wave
  const int lane = (int)(threadIdx.x & 63), kd = 64 * (int)(word % nmw) + lane;
  const SetsJob j{o, n_k, nx, ny, ncs, nmw, cst, mask};
  sets_word(j, word, lane, kd < n_k ? kc[kd] : make_double2(0.0, 0.0));
}

// chi(Kc) + theta and the counter reset, done by the interval-table kernel when kchi is given
struct ChiArgs {
  const float* theta;
  double* kchi;
  unsigned long long* stats;
  int groups;
};

static void launch_colsets(const double2* kc, int n_k, int nx, int ny, const Optics& o, int4* cst, uint64_t* cmask,
                           int nmw, hipStream_t s, const ChiArgs& chi = ChiArgs{}) {
  STEM_TRACE("ssb_colsets", s);
  const int B = 1024 / ny, ncs = (nx / 2 + 1 + B - 1) / B;
  const int64_t words = (int64_t)ncs * nmw;
  const int mask_blocks = (int)((words + 3) / 4);
  const int chi_blocks = chi.kchi ? (n_k + 255) / 256 : 0;
  hipLaunchKernelGGL(k_colsets, dim3((unsigned)(mask_blocks + chi_blocks)), dim3(256), 0, s, kc, n_k, nx, ny, o, B, ncs,
                     nmw, cst, cmask, mask_blocks, chi.theta, chi.kchi, chi.stats, chi.groups);
}

// chi identically zero (every monomial coefficient 0) and no per-pixel theta: the phase factors of
// Eq. 3 are all exactly 1
static int chi_is_zero(const Optics& o, const float* theta) {
  return !theta && o.p20 == 0.0 && o.p02 == 0.0 && o.p11 == 0.0 && o.p30 == 0.0 && o.p21 == 0.0 && o.p12 == 0.0 &&
         o.p03 == 0.0 && o.p4 == 0.0;
}

// the interval table and the active-pixel mask, then the fused column sum
// the interval table and the active-pixel mask (unless the x-stage built them: sets_ready), then
// the fused column sum; wcnt receives its pair count per wave
static int launch_yreduce(int prec, int ny, float2* X, const double2* kc, const double* kchi, int4* cst,
                          uint64_t* cmask, int nmw, int n_k, int nx, int ngroups, const Optics& o, int store_g,
                          int chi0, float2* part, unsigned long long* wcnt, hipStream_t s,
                          const ChiArgs& chi = ChiArgs{}, int sets_ready = 0) {
  if (!sets_ready) {
    launch_colsets(kc, n_k, nx, ny, o, cst, cmask, nmw, s, chi);
    STEM_LAUNCH_CHECK();
  }
  switch (prec) {
    case STEM_DFT_BF16_SPLIT:
      return launch_yreduce_p<STEM_DFT_BF16_SPLIT>(ny, X, kc, kchi, cst, cmask, nmw, n_k, nx, ngroups, o, store_g,
                                                   chi0, part, wcnt, s);
    case STEM_DFT_FP16_SPLIT:
      return launch_yreduce_p<STEM_DFT_FP16_SPLIT>(ny, X, kc, kchi, cst, cmask, nmw, n_k, nx, ngroups, o, store_g,
                                                   chi0, part, wcnt, s);
    default:
      return launch_yreduce_p<STEM_FFT_FP32>(ny, X, kc, kchi, cst, cmask, nmw, n_k, nx, ngroups, o, store_g, chi0,
                                             part, wcnt, s);
  }
}

// Eq. 3 from the stored G without normalisation (REFOCUS): the fused sum over the stored columns
static int launch_ysum_stored(int ny, float2* G, const double2* kc, const double* kchi, int4* cst, uint64_t* cmask,
                              int nmw, int n_k, int nx, int ngroups, const Optics& o, int chi0, float2* part,
                              unsigned long long* wcnt, hipStream_t s, const ChiArgs& chi) {
  launch_colsets(kc, n_k, nx, ny, o, cst, cmask, nmw, s, chi);
  STEM_LAUNCH_CHECK();
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  const dim3 grid((unsigned)(((ncs + 3) / 4) * ngroups)), blk(kYThreads);
  STEM_TRACE("ssb_reduce", s);
  const int st = with_n(ny, [&](auto nc) {
    using XF = XfNone<decltype(nc)::value>;
    if (chi0)
      hipLaunchKernelGGL((k_yreduce<XF, true>), grid, blk, 0, s, G, kc, kchi, cst, cmask, nmw, n_k, nx, ngroups, o,
                         0, part, wcnt);
    else
      hipLaunchKernelGGL((k_yreduce<XF, false>), grid, blk, 0, s, G, kc, kchi, cst, cmask, nmw, n_k, nx, ngroups, o,
                         0, part, wcnt);
  });
  if (st) return st;
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

static int launch_yadjoint(int prec, int ny, const float2* X, const double2* kc, const double* kchi, int4* cst,
                           uint64_t* cmask, int nmw, int n_k, int nx, int ngroups, const Optics& o, int g_stored,
                           const float2* Tbt, double* pdc, float* pdth, hipStream_t s, const ChiArgs& chi) {
  launch_colsets(kc, n_k, nx, ny, o, cst, cmask, nmw, s, chi);
  STEM_LAUNCH_CHECK();
  switch (prec) {
    case STEM_DFT_BF16_SPLIT:
      return launch_yadjoint_p<STEM_DFT_BF16_SPLIT>(ny, X, kc, kchi, cst, n_k, nx, ngroups, o, g_stored, Tbt, pdc,
                                                    pdth, s);
    case STEM_DFT_FP16_SPLIT:
      return launch_yadjoint_p<STEM_DFT_FP16_SPLIT>(ny, X, kc, kchi, cst, n_k, nx, ngroups, o, g_stored, Tbt, pdc,
                                                    pdth, s);
    default:
      return launch_yadjoint_p<STEM_FFT_FP32>(ny, X, kc, kchi, cst, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth,
                                              s);
  }
}

// ---------------------------------------------------------------------------------------------
// chi(Kc) + theta per kept pixel

__global__ void k_chi_table(const double2* __restrict__ kc, const float* __restrict__ theta, int n_k,
                            Optics o, double* __restrict__ kchi, unsigned long long* __restrict__ stats,
                            int groups) {
  const int kd = blockIdx.x * blockDim.x + threadIdx.x;
  if (kd < 4) stats[kd] = kd == 1 ? (unsigned long long)groups : 0ull;  // counters of the sum that follows
  if (kd >= n_k) return;
  const double2 k = kc[kd];
  kchi[kd] = chi_poly(k.x, k.y, o) + (theta ? (double)theta[kd] : 0.0);
}

// ---------------------------------------------------------------------------------------------
// Eq. 3 from a stored G: one thread per Q, Q in column-major order q = mx*Ny + my (a wave
// shares one column, so Qx is uniform).  Pixels are visited row by row of the kept set; a
// row with |Ky - Qy| >= r, or the rest of a row once Kx - Qx >= r, cannot satisfy |K - Q| < r
// under the same rounded arithmetic (|d| >= r implies fl(d*d) >= fl(r*r)), so skipping them
// leaves the set unchanged.

__global__ void __launch_bounds__(256) k_reduce(const float2* __restrict__ G, const RowRun* __restrict__ rows,
                                                int nby, const double2* __restrict__ kc,
                                                const double* __restrict__ kchi, int ny, int nx,
                                                Optics o, int normalize, float2* __restrict__ Tt,
                                                unsigned long long* __restrict__ stats) {
  const int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q0 < (int64_t)ny * nx;
  const int64_t q = valid ? q0 : 0;
  const int mx = (int)(q / ny), my = (int)(q % ny);
  const int ix = signed_index(mx, nx), iy = signed_index(my, ny);
  const double qx = (double)ix * o.sx;
  const double qy = (double)iy * o.sy;
  const bool mir = mx > nx / 2;
  const int gmx = mir ? nx - mx : mx, gmy = mir ? (ny - my) % ny : my;
  const int nh = nx / 2 + 1;
  const float2* gcol = G + (int64_t)gmx * ny + gmy;
  const int64_t kstride = (int64_t)nh * ny;
  float2 acc = make_float2(0.f, 0.f);
  int cnt = 0;
  for (int by = 0; by < nby; ++by) {
    const RowRun rr = rows[by];
    if (rr.hi <= rr.lo) continue;
    const double ky = kc[rr.start].y;
    if (!(valid && fabs(ky - qy) < o.r)) continue;
    for (int kd = rr.start; kd < rr.start + (rr.hi - rr.lo); ++kd) {
      const double kx = kc[kd].x;
      if (kx - qx >= o.r) break;
      if (qx - kx >= o.r) continue;
      if (!overlap_screened(kx, ky, (float)kx, (float)ky, ix, iy, o)) continue;
      const double psi = chi_poly(kx - qx, ky - qy, o) - kchi[kd];
      float2 g = gcol[kd * kstride];
      if (mir) g = cconj(g);
      const float2 e = expi_reduced(psi);
      acc.x += g.x * e.x - g.y * e.y;
      acc.y += g.x * e.y + g.y * e.x;
      ++cnt;
    }
  }
  if (normalize && cnt > 0) acc = cscale(acc, 1.f / (float)cnt);
  if (valid) Tt[q] = acc;
  // number of double-overlap pairs of this sum, one atomic per wave
  unsigned long long c = valid ? (unsigned long long)cnt : 0ull;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(stats, c);
}

// number of pixel groups of the fused sum: about 4096 waves, at most n_k, partial sums <= 64 MB
static int yreduce_groups(int ny, int nx, int n_k) {
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  // about 2560 waves: 1.25 times the waves the GPU holds at once (256 CUs x 8 at this kernel's
  // register use), so that waves of cheap columns (few pixels with a non-empty set) free their
  // slots for the rest; measured at scan1024 (513 column sets): 5 groups 139 us, 4 groups 145 us,
  // 8 groups 156 us
  const int blocks_per_group = (ncs + 3) / 4;
  int g = (2560 + 2 * blocks_per_group) / (4 * blocks_per_group);
  const int64_t F = (int64_t)ny * nx;
  const int gmax = (int)((64ll << 20) / (F * 8));
  if (g > gmax) g = gmax;
  if (g > n_k) g = n_k;
  if (g < 1) g = 1;
  return g;
}

// T[mx][my] (column-major) -> d_T[my][mx] (row-major)
__global__ void k_transpose_T(const float2* __restrict__ Tt, int ny, int nx, float2* __restrict__ out) {
  __shared__ float2 tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx over my (rows of Tt are mx)
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int mx = by + j, my = bx + threadIdx.x;
    if (mx < nx && my < ny) tile[j][threadIdx.x] = Tt[(int64_t)mx * ny + my];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int my = bx + j, mx = by + threadIdx.x;
    if (mx < nx && my < ny) out[(int64_t)my * nx + mx] = tile[threadIdx.x][j];
  }
}

// ---------------------------------------------------------------------------------------------
// sums the adjoint partials in a fixed order: dL/dc over waves (workgroup 0), dL/dtheta over
// column sets (one thread per pixel, eight independent loads in flight)

__global__ void __launch_bounds__(256) k_adjoint_final(const double* __restrict__ pdc, int64_t npdc,
                                                       const float* __restrict__ pdth, int64_t npdth, int n_k,
                                                       double* __restrict__ dLdc, float* __restrict__ dLdth) {
  if (blockIdx.x == 0) {
    __shared__ double s[256][8];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < npdc; b += blockDim.x)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] += pdc[b * 8 + j];
#pragma unroll
    for (int j = 0; j < 8; ++j) s[threadIdx.x][j] = acc[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h)
#pragma unroll
        for (int j = 0; j < 8; ++j) s[threadIdx.x][j] += s[threadIdx.x + h][j];
      __syncthreads();
    }
    if (threadIdx.x < 8) dLdc[threadIdx.x] = s[0][threadIdx.x];
    return;
  }
  const int kd = (blockIdx.x - 1) * blockDim.x + threadIdx.x;
  if (!dLdth || kd >= n_k) return;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t b = 0;
  for (; b + 8 <= npdth; b += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)pdth[(b + u) * n_k + kd];
  for (; b < npdth; ++b) a[0] += (double)pdth[b * n_k + kd];
  dLdth[kd] = (float)(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
}

// ---------------------------------------------------------------------------------------------
// host helpers

static Optics make_optics(const stem_optics& op, const stem_scan& sc) {
  Optics o;
  o.lam = op.lam;
  o.dk = op.dk;
  o.r = op.r_bf;
  o.r2 = op.r_bf * op.r_bf;
  for (int j = 0; j < 8; ++j) o.c[j] = op.c[j];
  o.sx = 1.0 / (((double)sc.nx * sc.step) * op.dk);
  o.sy = 1.0 / (((double)sc.ny * sc.step) * op.dk);
  optics_poly(o);
  optics_screen(o, sc.ny, sc.nx);
  return o;
}

struct Bufs {
  RowRun* rows;
  double2* kc;
  double* kchi;
  int4* cst;
  uint64_t* cmask;
  int16_t* lut;
  unsigned long long* stats;
  void* D;
  float2* X;
  float2* T;
  float2* A;
  float2* Tb;
  double* pdc;
  float* pdth;
  float2* part;
  unsigned long long* wcnt;  // pair counts per wave of the fused sum
};

static Bufs carve(void* state, const SsbLayout& L) {
  char* p = (char*)state;
  return Bufs{(RowRun*)(p + L.rows), (double2*)(p + L.kc), (double*)(p + L.kchi), (int4*)(p + L.cst),
              (uint64_t*)(p + L.cmask), (int16_t*)(p + L.lut),
              (unsigned long long*)(p + L.stats), (void*)(p + L.D),
              (float2*)(p + L.X),    (float2*)(p + L.T),  (float2*)(p + L.A),     (float2*)(p + L.Tb),
              (double*)(p + L.pdc),  (float*)(p + L.pdth), (float2*)(p + L.part),
              (unsigned long long*)(p + L.wcnt)};
}

static int check_common(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                        const stem_ssb* ssb, int* n_k) {
  if (!det_ok(det) || !scan || !optics_ok(optics) || !ssb) return STEM_EINVAL;
  if (!is_pow2_in(scan->ny, 32, 1024) || !is_pow2_in(scan->nx, 32, 1024) || !(scan->step > 0))
    return STEM_EINVAL;
  if (ssb->d_bits != 8 && ssb->d_bits != 16) return STEM_EINVAL;
  if (ssb->precision != STEM_FFT_FP32 && ssb->precision != STEM_DFT_BF16_SPLIT &&
      ssb->precision != STEM_DFT_FP16_SPLIT)
    return STEM_EINVAL;
  if (ssb->g_mode != STEM_G_STORE && ssb->g_mode != STEM_G_RECOMPUTE) return STEM_EINVAL;
  const int n = count_pixels(*det, optics->r_bf * optics->r_bf);
  if (n <= 0 || n > kMaxPixels) return STEM_EINVAL;
  *n_k = n;
  return STEM_OK;
}

// T = sum of the partial sums (column-major [mx][my]); phi = Im IFFT2(T); d_T row-major.
static int run_phase(const SsbLayout& L, const Bufs& b, const stem_scan& sc, const float2* parts, int nparts,
                     float* d_phase, float* d_T, hipStream_t s) {
  const int ny = sc.ny, nx = sc.nx;
  RowFftArgs a{};
  // inverse along my of each mx row of T -> A[ry][mx]; the summed T is kept in the state
  a.nrows = nx;
  a.in_c = parts;
  a.nparts = nparts;
  a.part_stride = L.F;
  a.sum_out = parts == b.T ? nullptr : b.T;
  a.out_c = b.A;
  a.out_stride = nx;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "phase_fft";
  if (parts == b.part) {
    // the fused sum's pair counts per wave become the state's counters
    a.wcnt = b.wcnt;
    a.nwcnt = L.nwy;
    a.stats = b.stats;
    a.stats_groups = nparts;
  }
  int st = launch_row_fft(ny, true, IN_C64_SUM, OUT_T_C64, a, s);
  if (st) return st;
  if (d_phase) {
    a = RowFftArgs{};
    a.nrows = ny;
    a.in_c = b.A;
    a.out_f = d_phase;
    a.osc = make_float2((float)(1.0 / (double)L.F), 0.f);
    a.tag = "phase_fft";
    if ((st = launch_row_fft(nx, true, IN_C64, OUT_ROW_IM, a, s))) return st;
  }
  if (d_T) {
    STEM_TRACE("t_transpose", s);
    hipLaunchKernelGGL(k_transpose_T, dim3((ny + 31) / 32, (nx + 31) / 32), dim3(32, 8), 0, s, b.T, ny, nx,
                       (float2*)d_T);
    STEM_LAUNCH_CHECK();
  }
  return STEM_OK;
}

static int run_chi_table(const Bufs& b, const float* d_theta, int n_k, const Optics& o, int groups,
                         hipStream_t s) {
  STEM_TRACE("chi_table", s);
  hipLaunchKernelGGL(k_chi_table, dim3((n_k + 255) / 256), dim3(256), 0, s, b.kc, d_theta, n_k, o, b.kchi,
                     b.stats, groups);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

static int run_reduce_stored(const SsbLayout& L, const Bufs& b, int ny, int nx, const Optics& o, int normalize,
                             hipStream_t s) {
  STEM_TRACE("ssb_reduce", s);
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)L.nblk), dim3(256), 0, s, b.X, b.rows, L.nby, b.kc, b.kchi, ny, nx,
                     o, normalize, b.T, b.stats);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem

// ---------------------------------------------------------------------------------------------
// C ABI

using namespace stem;

extern "C" int ssb_num_pixels(const stem_det* det, const stem_optics* optics) {
  if (!det_ok(det) || !optics_ok(optics)) return -STEM_EINVAL;
  return count_pixels(*det, optics->r_bf * optics->r_bf);
}

extern "C" size_t ssb_state_bytes(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                                  const stem_ssb* ssb) {
  int n_k;
  if (check_common(det, scan, optics, ssb, &n_k)) return 0;
  SsbLayout L;
  return make_layout(*det, *scan, *ssb, n_k, &L);
}

extern "C" int ssb_state_region(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                                const stem_ssb* ssb, int region, size_t* offset, size_t* bytes) {
  int n_k;
  if (check_common(det, scan, optics, ssb, &n_k) || !offset || !bytes) return STEM_EINVAL;
  SsbLayout L;
  make_layout(*det, *scan, *ssb, n_k, &L);
  switch (region) {
    case STEM_REGION_D: *offset = L.D; *bytes = (size_t)n_k * L.F * (ssb->d_bits / 8); break;
    case STEM_REGION_G: *offset = L.X; *bytes = (size_t)n_k * L.nh * scan->ny * sizeof(float2); break;
    case STEM_REGION_T: *offset = L.T; *bytes = (size_t)L.F * sizeof(float2); break;
    case STEM_REGION_KC: *offset = L.kc; *bytes = (size_t)n_k * sizeof(double2); break;
    case STEM_REGION_STATS: *offset = L.stats; *bytes = 4 * sizeof(unsigned long long); break;
    default: return STEM_EINVAL;
  }
  return STEM_OK;
}

static int reconstruct(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                       const stem_det* det, const stem_scan* scan, const stem_optics* optics, const stem_ssb* ssb,
                       int mode, const float* d_theta, void* state, size_t state_bytes, float* d_phase, float* d_T,
                       const ComOut* com, int32_t* d_status, void* stream_) {
  int n_k;
  int st = check_common(det, scan, optics, ssb, &n_k);
  if (st) return st;
  if (mode < STEM_SSB_ACCUMULATE || mode > STEM_SSB_ONESHOT) return STEM_EINVAL;
  SsbLayout L;
  make_layout(*det, *scan, *ssb, n_k, &L);
  if (!state || ((uintptr_t)state & 255) || state_bytes < L.total) return STEM_EWORKSPACE;
  if (mode == STEM_SSB_REFOCUS && ssb->g_mode != STEM_G_STORE) return STEM_ESTATE;
  hipStream_t s = (hipStream_t)stream_;
  const Bufs b = carve(state, L);
  const int ny = scan->ny, nx = scan->nx;
  const Optics o = make_optics(*optics, *scan);

  if (mode == STEM_SSB_ACCUMULATE || mode == STEM_SSB_ONESHOT) {
    if (mode == STEM_SSB_ONESHOT) {
      frame0 = 0;
      n_frames = L.F;
    }
    if (!d_idx || !d_off) return STEM_EINVAL;
    if (frame0 < 0 || n_frames <= 0 || frame0 % nx || n_frames % nx || frame0 + n_frames > L.F)
      return STEM_EINVAL;
    // the binning also builds the interval table and the active-pixel mask when it can (geometry only)
    const SetsJob job{o, n_k, nx, ny, L.ncs, L.nmw, b.cst, b.cmask};
    if ((st = launch_bin(d_idx, d_off, frame0, n_frames, *det, o.r2, b.rows, b.kc, b.lut, n_k, L.F, b.D,
                          ssb->d_bits, d_status, s, com, &job)))
      return st;
    const int ry0 = (int)(frame0 / nx), nr = (int)(n_frames / nx);
    const int64_t nrows = (int64_t)n_k * nr;
    if (ssb->d_bits == 8)
      st = launch_xstage_t<uint8_t>(ssb->precision, nx, (const uint8_t*)b.D, ny, ry0, nr, nrows, b.X, s);
    else
      st = launch_xstage_t<uint16_t>(ssb->precision, nx, (const uint16_t*)b.D, ny, ry0, nr, nrows, b.X, s);
    if (st) return st;
    if (mode == STEM_SSB_ACCUMULATE) return STEM_OK;
  }
  // without normalisation chi(Kc) + theta comes with the interval table of the fused sum
  const ChiArgs chi{d_theta, b.kchi, b.stats, L.groups};
  if (ssb->normalize && (st = run_chi_table(b, d_theta, n_k, o, 1, s))) return st;
  if (mode == STEM_SSB_REFOCUS) {
    // Eq. 3 again from the stored G: per-Q normalised sum, or the fused sum over stored columns
    if (ssb->normalize) {
      if ((st = run_reduce_stored(L, b, ny, nx, o, 1, s))) return st;
      return run_phase(L, b, *scan, b.T, 1, d_phase, d_T, s);
    }
    if ((st = launch_ysum_stored(ny, b.X, b.kc, b.kchi, b.cst, b.cmask, L.nmw, n_k, nx, L.groups, o,
                                 chi_is_zero(o, d_theta), b.part, b.wcnt, s, chi)))
      return st;
    return run_phase(L, b, *scan, b.part, L.groups, d_phase, d_T, s);
  }
  if (ssb->normalize && ssb->precision != STEM_FFT_FP32) {
    // split precision: the fused kernel transforms X -> G in place (its partial sums are not
    // used); the counters are reset before the per-Q normalised sum
    if ((st = launch_yreduce(ssb->precision, ny, b.X, b.kc, b.kchi, b.cst, b.cmask, L.nmw, n_k, nx, L.groups, o, 1,
                             1, b.part, b.wcnt, s)))
      return st;
    if ((st = run_chi_table(b, d_theta, n_k, o, 1, s))) return st;
    if ((st = run_reduce_stored(L, b, ny, nx, o, 1, s))) return st;
    return run_phase(L, b, *scan, b.T, 1, d_phase, d_T, s);
  }
  if (ssb->normalize) {
    // the normalised sum needs each Q's pair count over all pixels: column transform in place
    // (X -> G), then the per-Q sum
    RowFftArgs a{};
    a.nrows = (int64_t)n_k * L.nh;
    a.in_c = b.X;
    a.out_c = b.X;
    a.osc = make_float2(1.f, 0.f);
    a.tag = "ystage_fft";
    if ((st = launch_row_fft(ny, false, IN_C64, OUT_ROW_C64, a, s))) return st;
    if ((st = run_reduce_stored(L, b, ny, nx, o, 1, s))) return st;
    return run_phase(L, b, *scan, b.T, 1, d_phase, d_T, s);
  }
  // without aberrations the sum needs only the interval table and the mask, which ACCUMULATE's
  // binning built (when it bins through its LDS table); otherwise the table kernel also tabulates
  // chi(Kc) + theta
  const int chi0 = chi_is_zero(o, d_theta);
  const int sets_ready = chi0 && bin_builds_sets(*det, o.r2);
  if ((st = launch_yreduce(ssb->precision, ny, b.X, b.kc, b.kchi, b.cst, b.cmask, L.nmw, n_k, nx, L.groups, o,
                           ssb->g_mode == STEM_G_STORE, chi0, b.part, b.wcnt, s, chi, sets_ready)))
    return st;
  return run_phase(L, b, *scan, b.part, L.groups, d_phase, d_T, s);
}

extern "C" int ssb_reconstruct(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                               const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                               const stem_ssb* ssb, int mode, const float* d_theta, void* state,
                               size_t state_bytes, float* d_phase, float* d_T, int32_t* d_status,
                               void* stream_) {
  return reconstruct(d_idx, d_off, frame0, n_frames, det, scan, optics, ssb, mode, d_theta, state, state_bytes,
                     d_phase, d_T, nullptr, d_status, stream_);
}

extern "C" int ssb_reconstruct_com(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                                   const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                                   const stem_ssb* ssb, int mode, const float* d_theta, void* state,
                                   size_t state_bytes, float* d_phase, float* d_T, double* d_com64,
                                   float* d_com32, int32_t* d_counts, int32_t* d_status, void* stream_) {
  if (mode != STEM_SSB_ACCUMULATE && mode != STEM_SSB_ONESHOT) return STEM_EINVAL;
  if (!d_com64 && !d_com32 && !d_counts) return STEM_EINVAL;
  if (!det || det->W >= 65536 || det->H >= 65536) return STEM_EINVAL;
  if (!scan) return STEM_EINVAL;
  const ComOut com{d_com64, d_com32, d_counts, (int64_t)scan->ny * scan->nx, det->cx, det->cy};
  return reconstruct(d_idx, d_off, frame0, n_frames, det, scan, optics, ssb, mode, d_theta, state, state_bytes,
                     d_phase, d_T, &com, d_status, stream_);
}

// ---------------------------------------------------------------------------------------------
// G(K, Q) at selected Q as binned detector images: one wave per (bin, Q)

struct PanelQ {
  int32_t my[STEM_MAX_PANEL], mx[STEM_MAX_PANEL];
};

__global__ void __launch_bounds__(64) k_g_panel(const float2* __restrict__ X, const RowRun* __restrict__ rows,
                                               int nbx, int n_k, int ny, int nx, PanelQ q, int g_stored,
                                               float2* __restrict__ img) {
  const int bin = blockIdx.x, j = blockIdx.y;  // bin = by * nbx + bx
  const int by = bin / nbx, bx = bin % nbx;
  const int lane = threadIdx.x;
  float2* out = img + (int64_t)j * gridDim.x + bin;
  const RowRun rr = rows[by];
  if (bx < rr.lo || bx >= rr.hi) {
    if (lane == 0) *out = make_float2(0.f, 0.f);
    return;
  }
  const int kd = rr.start + bx - rr.lo;
  if (kd < 0 || kd >= n_k) {  // a state whose geometry was never computed: nothing is read
    if (lane == 0) *out = make_float2(0.f, 0.f);
    return;
  }
  int my = q.my[j], mx = q.mx[j];
  const bool cj = 2 * mx > nx;  // G(K, Q) = conj G(K, -Q): read the half spectrum at -Q
  if (cj) {
    mx = nx - mx;
    my = (ny - my) & (ny - 1);
  }
  const float2* col = X + ((int64_t)kd * (nx / 2 + 1) + mx) * ny;
  float2 v;
  if (g_stored) {
    v = col[my];
  } else {
    // sum over ry of X exp(-2 pi i my ry / Ny), angles reduced exactly as integers mod Ny
    double re = 0.0, im = 0.0;
    for (int ry = lane; ry < ny; ry += 64) {
      const int k = (my * ry) & (ny - 1);
      double sn, cs;
      sincospi(2.0 * (double)k / (double)ny, &sn, &cs);
      const float2 x = col[ry];
      re += (double)x.x * cs + (double)x.y * sn;
      im += (double)x.y * cs - (double)x.x * sn;
    }
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    v = make_float2((float)re, (float)im);
  }
  if (cj) v.y = -v.y;
  if (lane == 0) *out = v;
}

extern "C" int ssb_g_panel(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                           const stem_ssb* ssb, const void* state, size_t state_bytes, int n_q,
                           const int32_t* h_my, const int32_t* h_mx, float* d_img, void* stream_) {
  int n_k;
  int st = check_common(det, scan, optics, ssb, &n_k);
  if (st) return st;
  if (!h_my || !h_mx || !d_img || n_q < 1 || n_q > STEM_MAX_PANEL) return STEM_EINVAL;
  PanelQ q{};
  for (int j = 0; j < n_q; ++j) {
    if (h_my[j] < 0 || h_my[j] >= scan->ny || h_mx[j] < 0 || h_mx[j] >= scan->nx) return STEM_EINVAL;
    q.my[j] = h_my[j];
    q.mx[j] = h_mx[j];
  }
  SsbLayout L;
  make_layout(*det, *scan, *ssb, n_k, &L);
  if (!state || ((uintptr_t)state & 255) || state_bytes < L.total) return STEM_EWORKSPACE;
  const Bufs b = carve(const_cast<void*>(state), L);
  const int nbx = det->W / det->bin, nby = det->H / det->bin;
  hipStream_t s = (hipStream_t)stream_;
  STEM_TRACE("g_panel", s);
  hipLaunchKernelGGL(k_g_panel, dim3((unsigned)(nbx * nby), (unsigned)n_q), dim3(64), 0, s, b.X, b.rows, nbx, n_k,
                     scan->ny, scan->nx, q, ssb->g_mode == STEM_G_STORE ? 1 : 0, (float2*)d_img);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

extern "C" int ssb_backward(const float* d_dLdphi, const stem_det* det, const stem_scan* scan,
                            const stem_optics* optics, const stem_ssb* ssb, const float* d_theta, void* state,
                            size_t state_bytes, double* d_dLdc, float* d_dLdtheta, int32_t* d_status,
                            void* stream_) {
  (void)d_status;
  int n_k;
  int st = check_common(det, scan, optics, ssb, &n_k);
  if (st) return st;
  if (!d_dLdphi || !d_dLdc || ssb->normalize) return STEM_EINVAL;
  SsbLayout L;
  make_layout(*det, *scan, *ssb, n_k, &L);
  if (!state || ((uintptr_t)state & 255) || state_bytes < L.total) return STEM_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream_;
  const Bufs b = carve(state, L);
  const int ny = scan->ny, nx = scan->nx;
  const Optics o = make_optics(*optics, *scan);
  // Tbar = (i/N_R) FFT2(gbar), column-major [mx][my]
  RowFftArgs a{};
  a.nrows = ny;
  a.in_f0 = d_dLdphi;
  a.s0 = 1.f;
  a.out_c = b.A;
  a.out_stride = ny;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "adj_fft";
  if ((st = launch_row_fft(nx, false, IN_F32_PAIR, OUT_T_C64, a, s))) return st;
  a = RowFftArgs{};
  a.nrows = nx;
  a.in_c = b.A;
  a.out_c = b.Tb;
  a.osc = make_float2(0.f, (float)(1.0 / (double)L.F));
  a.tag = "adj_fft";
  if ((st = launch_row_fft(ny, false, IN_C64, OUT_ROW_C64, a, s))) return st;
  if ((st = launch_yadjoint(ssb->precision, ny, b.X, b.kc, b.kchi, b.cst, b.cmask, L.nmw, n_k, nx, L.groups, o,
                            ssb->g_mode == STEM_G_STORE, b.Tb, b.pdc, b.pdth, s,
                            ChiArgs{d_theta, b.kchi, b.stats, L.groups})))
    return st;
  {
    STEM_TRACE("ssb_adjoint_final", s);
    hipLaunchKernelGGL(k_adjoint_final, dim3(1 + (n_k + 255) / 256), dim3(256), 0, s, b.pdc, L.nwy, b.pdth,
                       (int64_t)L.ncs, n_k, d_dLdc, d_dLdtheta);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
