// Single-sideband (SSB) ptychography from linear-index events (Sec. IV) and its adjoint.
//
// Pipeline (state buffer owned by the caller):
//   k_bin          events -> D[kd][ry][rx] (uint8/uint16 counts), kept-set geometry     (Table 1)
//   k_xstage       real row FFT along rx, output transposed X[kd][mx][ry], mx in [0, Nx/2]
//   k_yreduce      FFT along ry of every (kd, mx) column in registers (G, Eq. 2) fused with
//                  Eq. 3 over the double-overlap set -> partial sums of T per pixel group
//   phase          two inverse row FFT passes -> phi = Im IFFT2(T)
// The other half of the Q plane (mx > Nx/2) uses G(K, Q) = conj G(K, -Q) of the real input.
//
// G modes.  STEM_G_STORE keeps X for every pixel (written during ACCUMULATE) and, at FINALIZE,
// the double-overlap values of G (the pruned array, 8 bytes per pair): REFOCUS and the adjoint
// read only those.  STEM_G_RECOMPUTE keeps D only; every sum (and the adjoint) re-runs the row
// transform for a chunk of pixels at a time into a bounded scratch and fuses the column
// transform and the sum on it.
#include "common.h"
#include "fft_generic.h"
#include "fft_wave.h"
#include "ssb_fused.h"
#include "ssb_pruned.h"
#include "kernels.h"
#include "optics.h"
#include "trace.h"

namespace stem {

constexpr int kMaxPixels = 4096;
constexpr int kDefaultScratchMib = 64;  // row-transformed columns held at once in STEM_G_RECOMPUTE
#ifndef STEM_PRUNED_BLOCKS
#define STEM_PRUNED_BLOCKS 3072
#endif
constexpr int kPrunedBlocks = STEM_PRUNED_BLOCKS;  // (column, pixel group) items without a schedule

struct SsbLayout {
  int n_k, nby, nh;
  int64_t F;
  bool store;     // STEM_G_STORE
  int xpix;       // pixels whose row-transformed columns the X region holds (n_k, or one chunk)
  int ypix;       // pixels of the column-transform scratch (stored G of the other lengths), or 0
  int nchunks;    // pixel chunks of a sum
  int64_t pcap;   // entries of the pruned G array (0 without STEM_G_STORE)
  size_t rows, kc, kchi, cst, cmask, lut, stats, npq, D, X, Y, poff, ptot, pg, T, A, Tb, pdc, pdth, part, wcnt, pws, pcs,
      total;
  int nmw;      // 64-bit words per column set of the active-pixel mask
  int groups;   // pixel groups of the fused column kernels (the same for every chunk)
  int pgroups;  // pixel groups of the kernels over the stored double-overlap values
  int ncs;      // column sets (colset_width(Ny) half-spectrum columns each)
  bool fast;    // both scan lengths taken by the fused kernels (powers of two in [32, 1024])
  int64_t nwy;  // waves of the fused kernels
  int64_t nwp;  // waves of the refocus sum over the full columns of G (other scan lengths)
  int64_t nws;  // pieces the refocus sum over the stored values aims at
  int64_t nwq;  // STEM_G_STORE: waves (at most) of the refocus sum over the stored values
  int64_t part_rows;  // rows of Ny values the partial-sum buffer holds
  int64_t nwa;  // dL/dc partials of the adjoint over the stored values (one per workgroup)
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

// Upper bound of the double-overlap values of one pixel: the scan frequencies Q = (ix sx, iy sy)
// with |K - Q| < r.  The lattice cells around those points are disjoint and lie inside the disk of
// radius r + d (d the cell's half diagonal), so they number at most pi (r + d)^2 / (sx sy).
static int64_t pruned_bound(const stem_scan& scan, const stem_optics& op, int n_k) {
  const double sx = 1.0 / (((double)scan.nx * scan.step) * op.dk);
  const double sy = 1.0 / (((double)scan.ny * scan.step) * op.dk);
  const double d = 0.5 * __builtin_sqrt(sx * sx + sy * sy);
  const double r = op.r_bf * (1.0 + 1e-9) + d;
  const double F = (double)scan.ny * scan.nx;
  double per = __builtin_floor(3.14159265358979323846 * r * r / (sx * sy)) + 1.0;
  if (per > F) per = F;
  return (int64_t)per * n_k;
}

static size_t make_layout(const stem_det& det, const stem_scan& scan, const stem_optics& op, const stem_ssb& ssb,
                          int n_k, SsbLayout* L) {
  L->n_k = n_k;
  L->nby = det.H / det.bin;
  L->nh = scan.nx / 2 + 1;
  L->F = (int64_t)scan.ny * scan.nx;
  L->store = ssb.g_mode == STEM_G_STORE;
  L->fast = fast_length(scan.ny) && fast_length(scan.nx);
  const size_t per_pixel = (size_t)L->nh * scan.ny * sizeof(float2);
  // chunks of pixels whose columns fit the scratch: balanced, of xpix or xpix - 1 pixels
  int chunk;
  {
    const size_t cap = (size_t)(ssb.scratch_mib > 0 ? ssb.scratch_mib : kDefaultScratchMib) << 20;
    int nc = (int)(cap / per_pixel);
    nc = nc < 1 ? 1 : nc > n_k ? n_k : nc;
    L->nchunks = (n_k + nc - 1) / nc;
    chunk = (n_k + L->nchunks - 1) / L->nchunks;
  }
  L->ypix = 0;
  if (L->store) {
    // every pixel's row transform; the other lengths also transform the columns in chunks into a
    // scratch of their own (the row transform stays for the panel of G)
    L->xpix = n_k;
    if (L->fast) L->nchunks = 1;
    else L->ypix = chunk;
    L->pcap = pruned_bound(scan, op, n_k);
  } else {
    L->xpix = chunk;
    L->pcap = 0;
  }
  size_t o = 0;
  L->rows = o;  o = align256(o + sizeof(RowRun) * L->nby);
  L->kc = o;    o = align256(o + sizeof(double2) * n_k);
  L->kchi = o;  o = align256(o + sizeof(double) * n_k);
  L->cst = o;   o = align256(o + sizeof(int4) * n_k * L->nh);
  L->nmw = (n_k + 63) / 64;
  {
    const int B = colset_width(scan.ny);
    L->ncs = (L->nh + B - 1) / B;
  }
  L->cmask = o; o = align256(o + sizeof(uint64_t) * (size_t)L->nmw * L->ncs);
  L->lut = o;   o = align256(o + sizeof(int16_t) * (size_t)det.W * det.H);
  // the counters of the last sum, then the mark a FINALIZE leaves (ready_tag)
  L->stats = o; o = align256(o + sizeof(unsigned long long) * 5);
  L->npq = o;   o = align256(o + sizeof(int32_t) * (size_t)L->F);
  L->D = o;     o = align256(o + (size_t)n_k * L->F * (ssb.d_bits / 8));
  L->X = o;     o = align256(o + (size_t)L->xpix * per_pixel);
  L->Y = o;     o = align256(o + (size_t)L->ypix * per_pixel);
  L->poff = o;  o = align256(o + (L->store ? sizeof(int64_t) * ((size_t)n_k * scan.nx + 1) : 0));
  L->ptot = o;  o = align256(o + (L->store ? sizeof(int64_t) * (size_t)scan.nx : 0));
  L->pg = o;    o = align256(o + sizeof(float2) * (size_t)L->pcap);
  L->T = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->A = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->Tb = o;    o = align256(o + (size_t)L->F * sizeof(float2));
  // pixel groups: the same for every chunk (the partial sums of a later chunk add to the same
  // waves' partials), so at most the smallest chunk's pixel count
  int g = yreduce_groups(scan.ny, scan.nx, n_k);
  const int smallest = n_k / L->nchunks;
  if (g > smallest) g = smallest;
  L->groups = g < 1 ? 1 : g;
  L->nwy = (int64_t)((L->ncs + 3) / 4) * 4 * L->groups;
  // the kernels over the stored values: a wave (refocus) or workgroup (adjoint) per column of the
  // whole plane and pixel group, about kPrunedBlocks of them, at most the fused kernels' partial
  // sums
  {
    int pg = (kPrunedBlocks + scan.nx - 1) / scan.nx;
    const int gmax = yreduce_groups(scan.ny, scan.nx, n_k);
    pg = pg > n_k ? n_k : pg;
    pg = pg > gmax ? gmax : pg;
    L->pgroups = pg < 1 ? 1 : pg;
    L->nwp = psum_launch_waves(scan.ny, scan.nx, L->pgroups);
    L->nwa = padj_partials(scan.nx, L->pgroups);
    // the balanced pieces: as many as the GPU holds waves at once (more, one per column with
    // pairs, when the columns outnumber them)
    const int w = psum_waves(scan.ny);
    const int64_t nws = psum_stream_waves(scan.ny);
    L->nws = nws;
    L->nwq = L->store ? ((nws > scan.nx ? nws : scan.nx) + w - 1) / w * w : 0;
  }
  int64_t nw = L->nwy > L->nwp ? L->nwy : L->nwp;
  nw = nw > L->nwq ? nw : L->nwq;
  nw = nw > L->nwa ? nw : L->nwa;
  const int rows = L->ncs > scan.nx ? L->ncs : scan.nx;
  const int parts = L->groups > L->pgroups ? L->groups : L->pgroups;
  L->pdc = o;   o = align256(o + (size_t)nw * 8 * sizeof(double));
  L->pdth = o;  o = align256(o + (size_t)rows * n_k * sizeof(float));
  // partials: the fused kernels' and the adjoint's planes, or one row of ny values per piece of
  // the refocus sum
  size_t part_rows = (size_t)parts * scan.nx;
  if (part_rows < (size_t)L->nwq) part_rows = (size_t)L->nwq;
  L->part_rows = (int64_t)part_rows;
  L->part = o;  o = align256(o + part_rows * scan.ny * sizeof(float2));
  L->wcnt = o;  o = align256(o + (size_t)nw * sizeof(unsigned long long));
  // the refocus sum's tables (STEM_G_STORE): per piece its first run and entries, per column
  L->pws = o;   o = align256(o + (size_t)L->nwq * sizeof(PieceTab));
  L->pcs = o;   o = align256(o + (L->store ? sizeof(int64_t) * stream_ctab_words(scan.nx) : 0));
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
// Workgroups past the mask's also tabulate chi(Kc) + theta per pixel when kchi is given.
__global__ void __launch_bounds__(256) k_colsets(const double2* __restrict__ kc, int n_k, int nx, int ny, Optics o,
                                                 int B, int ncs, int nmw, int4* __restrict__ cst,
                                                 uint64_t* __restrict__ mask, int mask_blocks,
                                                 const float* __restrict__ theta, double* __restrict__ kchi) {
  if ((int)blockIdx.x >= mask_blocks) {
    const int kd = (blockIdx.x - mask_blocks) * blockDim.x + threadIdx.x;
    if (kd < n_k) {
      const double2 k = kc[kd];
      kchi[kd] = chi_poly(k.x, k.y, o) + (theta ? (double)theta[kd] : 0.0);
    }
    return;
  }
  const int64_t word = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (word >= (int64_t)ncs * nmw) return;  // uniform across the wave
  const int lane = (int)(threadIdx.x & 63), kd = 64 * (int)(word % nmw) + lane;
  const SetsJob j{o, n_k, nx, ny, ncs, nmw, cst, mask, B};
  sets_word(j, word, lane, kd < n_k ? kc[kd] : make_double2(0.0, 0.0));
}

// the interval table and mask, and chi(Kc) + theta when kchi is given
static int launch_colsets(const double2* kc, int n_k, int nx, int ny, const Optics& o, int4* cst, uint64_t* cmask,
                          int nmw, hipStream_t s, const float* theta, double* kchi) {
  STEM_TRACE("ssb_colsets", s);
  const int B = colset_width(ny), ncs = (nx / 2 + 1 + B - 1) / B;
  const int64_t words = (int64_t)ncs * nmw;
  const int mask_blocks = (int)((words + 3) / 4);
  const int chi_blocks = kchi ? (n_k + 255) / 256 : 0;
  hipLaunchKernelGGL(k_colsets, dim3((unsigned)(mask_blocks + chi_blocks)), dim3(256), 0, s, kc, n_k, nx, ny, o, B,
                     ncs, nmw, cst, cmask, mask_blocks, theta, kchi);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// chi identically zero (every monomial coefficient 0) and no per-pixel theta: the phase factors of
// Eq. 3 are all exactly 1
static int chi_is_zero(const Optics& o, const float* theta) {
  return !theta && o.p20 == 0.0 && o.p02 == 0.0 && o.p11 == 0.0 && o.p30 == 0.0 && o.p21 == 0.0 && o.p12 == 0.0 &&
         o.p03 == 0.0 && o.p4 == 0.0;
}

// the fused sum with the transform of precision prec (prec < 0: from the pruned G)
static int launch_yreduce(int prec, int ny, const YArgs& a, const Optics& o, int chi0, int pwrite, hipStream_t s) {
  switch (prec) {
    case STEM_DFT_BF16_SPLIT: return launch_yreduce_p<STEM_DFT_BF16_SPLIT>(ny, a, o, chi0, pwrite, s);
    case STEM_DFT_FP16_SPLIT: return launch_yreduce_p<STEM_DFT_FP16_SPLIT>(ny, a, o, chi0, pwrite, s);
    default: return launch_yreduce_p<STEM_FFT_FP32>(ny, a, o, chi0, pwrite, s);
  }
}

static int launch_yadjoint(int prec, int ny, const YArgs& a, const Optics& o, hipStream_t s) {
  switch (prec) {
    case STEM_DFT_BF16_SPLIT: return launch_yadjoint_p<STEM_DFT_BF16_SPLIT>(ny, a, o, s);
    case STEM_DFT_FP16_SPLIT: return launch_yadjoint_p<STEM_DFT_FP16_SPLIT>(ny, a, o, s);
    default: return launch_yadjoint_p<STEM_FFT_FP32>(ny, a, o, s);
  }
}

// ---------------------------------------------------------------------------------------------
// chi(Kc) + theta per kept pixel

__global__ void k_chi_table(const double2* __restrict__ kc, const float* __restrict__ theta, int n_k,
                            Optics o, double* __restrict__ kchi) {
  const int kd = blockIdx.x * blockDim.x + threadIdx.x;
  if (kd >= n_k) return;
  const double2 k = kc[kd];
  kchi[kd] = chi_poly(k.x, k.y, o) + (theta ? (double)theta[kd] : 0.0);
}

// ---------------------------------------------------------------------------------------------
// Number of double-overlap pixels of every scan frequency (the divisor of the normalised sum),
// column-major [mx][my] like T: one thread per Q, membership from the interval table (the set of
// column mx > Nx/2 is the mirror set of column Nx - mx).

__global__ void __launch_bounds__(256) k_pair_count(const int4* __restrict__ cst, int n_k, int ny, int nx,
                                                    int32_t* __restrict__ npq) {
  const int64_t F = (int64_t)ny * nx;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= F) return;
  const int mx = (int)(q / ny), my = (int)(q % ny);
  const int nc = nx / 2 + 1;
  const bool mir = 2 * mx > nx;
  const int c = mir ? nx - mx : mx;
  const int iy = signed_index(my, ny);
  int cnt = 0;
  int kd = 0;
  for (; kd + 4 <= n_k; kd += 4) {
    ColSet d[4], m[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_colsets(cst, (int64_t)(kd + u) * nc + c, d[u], m[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) cnt += (mir ? m[u] : d[u]).has(iy) ? 1 : 0;
  }
  for (; kd < n_k; ++kd) {
    ColSet d, m;
    load_colsets(cst, (int64_t)kd * nc + c, d, m);
    cnt += (mir ? m : d).has(iy) ? 1 : 0;
  }
  npq[q] = cnt;
}

// Offsets of the pruned double-overlap array: poff[mx * n_k + kd] = number of values of the
// (column, pixel) pairs before it in column-major, pixel-minor order; poff[Nx * n_k] = the total.
// Three passes: the runs of each column scanned by its own workgroup (offsets relative to the
// column, column totals to ptot), the column totals scanned by one workgroup, then each column's
// base added.

__device__ __forceinline__ int64_t pruned_size(const int4* __restrict__ cst, int kd, int mx, int nx) {
  const int nc = nx / 2 + 1;
  const bool mir = 2 * mx > nx;
  ColSet d, m;
  load_colsets(cst, (int64_t)kd * nc + (mir ? nx - mx : mx), d, m);
  return set_size(mir ? m : d);
}

// inclusive scan of one value per thread over a 256-thread workgroup (s: 256 entries)
__device__ __forceinline__ int64_t block_scan256(int64_t v, int64_t* s) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t u = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += u;
    __syncthreads();
  }
  const int64_t r = s[t];
  __syncthreads();
  return r;
}

// The first pass also writes the column's entry of the refocus sum's column table (ctab, see
// ssb_pruned.h): its cost and the span of its runs with entries.
__global__ void __launch_bounds__(256) k_prune_runs(const int4* __restrict__ cst, int n_k, int nx,
                                                    int64_t* __restrict__ poff, int64_t* __restrict__ ptot,
                                                    int64_t* __restrict__ ctab) {
  __shared__ int64_t s[256];
  const int mx = blockIdx.x;
  const int per = (n_k + 255) / 256;  // consecutive pixels per thread
  const int k0 = threadIdx.x * per;
  int64_t sum = 0, cost = 0;
  int lo = n_k, hi = -1;
  for (int kd = k0; kd < k0 + per && kd < n_k; ++kd) {
    const int64_t len = pruned_size(cst, kd, mx, nx);
    sum += len;
    if (len > 0) {
      cost += len + kRunCost;
      lo = min(lo, kd);
      hi = max(hi, kd);
    }
  }
  int64_t base = block_scan256(sum, s) - sum;
  for (int kd = k0; kd < k0 + per && kd < n_k; ++kd) {
    poff[(int64_t)mx * n_k + kd] = base;
    base += pruned_size(cst, kd, mx, nx);
  }
  if (threadIdx.x == 255) ptot[mx] = base;
  // the column's cost and span: wave reductions, then the four waves' in LDS
  for (int off = 32; off > 0; off >>= 1) {
    cost += __shfl_xor(cost, off);
    lo = min(lo, __shfl_xor(lo, off));
    hi = max(hi, __shfl_xor(hi, off));
  }
  __shared__ int64_t s_cost[4];
  __shared__ int s_lh[4][2];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_cost[w] = cost;
    s_lh[w][0] = lo;
    s_lh[w][1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int l = min(min(s_lh[0][0], s_lh[1][0]), min(s_lh[2][0], s_lh[3][0]));
    const int h = max(max(s_lh[0][1], s_lh[1][1]), max(s_lh[2][1], s_lh[3][1]));
    const int64_t r0 = (int64_t)mx * n_k;
    int64_t* col = ctab + (nx + 2) + 3 * (int64_t)mx;
    col[0] = (s_cost[0] + s_cost[1]) + (s_cost[2] + s_cost[3]);
    col[1] = h >= 0 ? r0 + l : 0;
    col[2] = h >= 0 ? r0 + h + 1 : 0;
  }
}

__global__ void __launch_bounds__(256) k_prune_bases(int n_k, int nx, int64_t* __restrict__ poff,
                                                     int64_t* __restrict__ ptot, int64_t pcap,
                                                     int32_t* __restrict__ status) {
  __shared__ int64_t s[256];
  const int per = (nx + 255) / 256;
  const int m0 = threadIdx.x * per;
  int64_t sum = 0;
  for (int mx = m0; mx < m0 + per && mx < nx; ++mx) sum += ptot[mx];
  int64_t base = block_scan256(sum, s) - sum;
  for (int mx = m0; mx < m0 + per && mx < nx; ++mx) {
    const int64_t t = ptot[mx];
    ptot[mx] = base;  // now the column's first entry
    base += t;
  }
  if (threadIdx.x == 255) {
    poff[(int64_t)nx * n_k] = base;
    if (base > pcap) report(status, STEM_EWORKSPACE);  // never with the layout's bound
  }
}

__global__ void __launch_bounds__(256) k_prune_add(int n_k, int64_t* __restrict__ poff,
                                                   const int64_t* __restrict__ ptot) {
  const int mx = blockIdx.x;
  const int64_t b = ptot[mx];
  for (int kd = threadIdx.x; kd < n_k; kd += 256) poff[(int64_t)mx * n_k + kd] += b;
}

// number of pixel groups of the fused sum: about 4096 waves, at most n_k, partial sums <= 64 MB
#ifndef STEM_YREDUCE_WAVES
#define STEM_YREDUCE_WAVES 2560
#endif

static int yreduce_groups(int ny, int nx, int n_k) {
  const int B = colset_width(ny);
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  // about 2560 waves: 1.25 times the waves the GPU holds at once (256 CUs x 8 at this kernel's
  // register use), so that waves of cheap columns (few pixels with a non-empty set) free their
  // slots for the rest; measured at scan1024 (513 column sets, no aberrations, each launch traced):
  // 3 groups 216-224 us, 4 groups 189-192, 5 groups 170-179, 6 groups 191-193, 7 groups 196-199,
  // 8 groups 188-191
  const int blocks_per_group = (ncs + 3) / 4;
  int g = (STEM_YREDUCE_WAVES + 2 * blocks_per_group) / (4 * blocks_per_group);
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
// sums the adjoint partials in a fixed order: dL/dc component j over the waves' partials
// (workgroup j < 8: a strided share per thread with four accumulators, then a tree over the
// workgroup), dL/dtheta over the npdth rows of partials (one wave per pixel: lane l takes rows
// l, l + 64, ..., then a fixed tree over the lanes)
constexpr int kFinalDcBlocks = 8;

__global__ void __launch_bounds__(256) k_adjoint_final(const double* __restrict__ pdc, int64_t npdc,
                                                       const float* __restrict__ pdth, int64_t npdth, int n_k,
                                                       const int64_t* __restrict__ pieces,
                                                       double* __restrict__ dLdc, float* __restrict__ dLdth) {
  if (blockIdx.x < kFinalDcBlocks) {
    __shared__ double s[256];
    const int j = blockIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t b = threadIdx.x;
    for (; b + 768 < npdc; b += 1024) {
      a0 += pdc[b * 8 + j];
      a1 += pdc[(b + 256) * 8 + j];
      a2 += pdc[(b + 512) * 8 + j];
      a3 += pdc[(b + 768) * 8 + j];
    }
    for (; b < npdc; b += 256) a0 += pdc[b * 8 + j];
    s[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) dLdc[j] = s[0];
    return;
  }
  const int lane = threadIdx.x & 63;
  const int kd = (blockIdx.x - kFinalDcBlocks) * 4 + (threadIdx.x >> 6);
  if (!dLdth || kd >= n_k) return;  // uniform per wave
  double a0 = 0.0, a1 = 0.0;
  int64_t r = lane;
  // with pieces (the adjoint over the stored values): a column without pieces has no pairs and
  // its row of pdth is not written, it adds 0
  auto row = [&](int64_t q) -> double {
    return pieces && pieces[q + 1] == pieces[q] ? 0.0 : (double)pdth[q * n_k + kd];
  };
  for (; r + 64 < npdth; r += 128) {
    a0 += row(r);
    a1 += row(r + 64);
  }
  for (; r < npdth; r += 64) a0 += row(r);
  double v = a0 + a1;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane == 0) dLdth[kd] = (float)v;
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
  int32_t* npq;
  void* D;
  float2* X;
  float2* Y;
  int64_t* poff;
  int64_t* ptot;
  float2* pg;
  float2* T;
  float2* A;
  float2* Tb;
  double* pdc;
  float* pdth;
  float2* part;
  unsigned long long* wcnt;  // pair counts and loads per wave of the fused kernels
  PieceTab* pws;             // refocus sum: per piece its first run and entries
  int64_t* pcs;              // refocus sum: per column its first piece, cost and span of runs
};

// The value a FINALIZE leaves in the state's mark word: a constant mixed with the layout's size,
// so that a state prepared for another layout, or never finalized, does not show it by chance.
static unsigned long long ready_tag(const SsbLayout& L) {
  return 0x5ab3f1d2c4e5968bull ^ ((unsigned long long)L.total * 0x9e3779b97f4a7c15ull);
}

static Bufs carve(void* state, const SsbLayout& L) {
  char* p = (char*)state;
  return Bufs{(RowRun*)(p + L.rows), (double2*)(p + L.kc), (double*)(p + L.kchi), (int4*)(p + L.cst),
              (uint64_t*)(p + L.cmask), (int16_t*)(p + L.lut), (unsigned long long*)(p + L.stats),
              (int32_t*)(p + L.npq), (void*)(p + L.D), (float2*)(p + L.X), (float2*)(p + L.Y), (int64_t*)(p + L.poff),
              (int64_t*)(p + L.ptot), (float2*)(p + L.pg), (float2*)(p + L.T), (float2*)(p + L.A), (float2*)(p + L.Tb),
              (double*)(p + L.pdc), (float*)(p + L.pdth), (float2*)(p + L.part),
              (unsigned long long*)(p + L.wcnt), (PieceTab*)(p + L.pws), (int64_t*)(p + L.pcs)};
}

static int check_common(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                        const stem_ssb* ssb, int* n_k) {
  if (!det_ok(det) || !scan || !optics_ok(optics) || !ssb) return STEM_EINVAL;
  if (!scan_length_ok(scan->ny) || !scan_length_ok(scan->nx) || !(scan->step > 0)) return STEM_EINVAL;
  if (ssb->d_bits != 8 && ssb->d_bits != 16) return STEM_EINVAL;
  if (ssb->precision != STEM_FFT_FP32 && ssb->precision != STEM_DFT_BF16_SPLIT &&
      ssb->precision != STEM_DFT_FP16_SPLIT)
    return STEM_EINVAL;
  if (ssb->g_mode != STEM_G_STORE && ssb->g_mode != STEM_G_RECOMPUTE) return STEM_EINVAL;
  // the split-precision matrix-core transforms exist for the fused kernels' lengths only
  if (ssb->precision != STEM_FFT_FP32 && !(fast_length(scan->ny) && fast_length(scan->nx))) return STEM_EINVAL;
  if (ssb->normalize != 0 && ssb->normalize != 1) return STEM_EINVAL;
  if (ssb->scratch_mib < 0 || ssb->scratch_mib > (1 << 20)) return STEM_EINVAL;
  const int n = count_pixels(*det, optics->r_bf * optics->r_bf);
  if (n <= 0 || n > kMaxPixels) return STEM_EINVAL;
  *n_k = n;
  return STEM_OK;
}

static YArgs yargs(const SsbLayout& L, const Bufs& b, int nx) {
  YArgs a{};
  a.X = b.X;
  a.xk0 = 0;
  a.kc = b.kc;
  a.kchi = b.kchi;
  a.cst = b.cst;
  a.cmask = b.cmask;
  a.nmw = L.nmw;
  a.n_k = L.n_k;
  a.nx = nx;
  a.k0 = 0;
  a.k1 = L.n_k;
  a.ngroups = L.groups;
  a.accumulate = 0;
  a.pg = b.pg;
  a.pgw = b.pg;
  a.poff = L.store ? b.poff : nullptr;
  a.pcap = L.pcap;
  a.part = b.part;
  a.wcnt = b.wcnt;
  a.Tbt = b.Tb;
  a.pdc = b.pdc;
  a.pdth = b.pdth;
  return a;
}

// the check of refocus and adjoint calls: their sum kernels do nothing, and report STEM_ESTATE,
// on a state that no FINALIZE has marked
static void need_finalize(YArgs& a, const SsbLayout& L, const Bufs& b, int32_t* d_status) {
  a.ready = b.stats + 4;
  a.ready_tag = ready_tag(L);
  a.status = d_status;
}

// pixels [k0, k1) of chunk ch
static void chunk_range(const SsbLayout& L, int ch, int& k0, int& k1) {
  k0 = (int)((int64_t)L.n_k * ch / L.nchunks);
  k1 = (int)((int64_t)L.n_k * (ch + 1) / L.nchunks);
}

// row transform of the pixels [k0, k1) (all scan rows) into the X region
static int xstage_pixels(const SsbLayout& L, const Bufs& b, const stem_ssb& ssb, int ny, int nx, int k0, int k1,
                         hipStream_t s) {
  const int64_t nrows = (int64_t)(k1 - k0) * ny;
  if (ssb.d_bits == 8)
    return launch_xstage_t<uint8_t>(ssb.precision, nx, (const uint8_t*)b.D + (size_t)k0 * L.F, ny, 0, ny, nrows, b.X,
                                    s);
  return launch_xstage_t<uint16_t>(ssb.precision, nx, (const uint16_t*)b.D + (size_t)k0 * L.F, ny, 0, ny, nrows, b.X,
                                   s);
}

// The other scan lengths: row transform of the pixels [k0, k1) (all rows) into X by the generic
// FFT (one real row per transform), then the column transforms of those pixels, from src into dst
// (in place when equal).
static int xstage_generic(const SsbLayout& L, const Bufs& b, const stem_ssb& ssb, int ny, int nx, int k0, int k1,
                          hipStream_t s) {
  RowFftArgs a{};
  a.nrows = (int64_t)(k1 - k0) * ny;
  a.in_u = ssb.d_bits == 8 ? (const void*)((const uint8_t*)b.D + (size_t)k0 * L.F)
                           : (const void*)((const uint16_t*)b.D + (size_t)k0 * L.F);
  a.out_c = b.X;
  a.xrows = ny;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "xstage_fft";
  return launch_row_fft(nx, false, ssb.d_bits == 8 ? IN_U8 : IN_U16, OUT_X, a, s);
}

static int colfft_generic(const SsbLayout& L, int ny, int k0, int k1, const float2* src, float2* dst, hipStream_t s) {
  RowFftArgs a{};
  a.nrows = (int64_t)(k1 - k0) * L.nh;
  a.in_c = src;
  a.out_c = dst;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "ystage_fft";
  return launch_row_fft(ny, false, IN_C64, OUT_ROW_C64, a, s);
}

// T = sum of the partial sums (column-major [mx][my]), divided by the pair count of each Q when
// npq is given; phi = Im IFFT2(T); d_T row-major.  The fused kernels' per-wave counters become the
// state's counters.
// part_seg: the partials are the rows of the refocus sum's pieces (row mx of T adds rows
// part_seg[mx] .. part_seg[mx + 1] - 1 of b.part) instead of nparts planes
// mark: the call is a FINALIZE, and the first pass leaves ready_tag in the state's mark word
static int run_phase(const SsbLayout& L, const Bufs& b, const stem_scan& sc, int nparts, int64_t nwaves, int nchunks,
                     const int32_t* npq, float* d_phase, float* d_T, hipStream_t s, bool mark,
                     const int64_t* part_seg = nullptr) {
  const int ny = sc.ny, nx = sc.nx;
  RowFftArgs a{};
  // inverse along my of each mx row of T -> A[ry][mx]; the summed T is kept in the state
  a.nrows = nx;
  a.in_c = b.part;
  a.nparts = nparts;
  a.part_stride = L.F;
  a.part_seg = part_seg;
  a.part_seg_rows = L.part_rows;
  a.sum_out = b.T;
  a.norm_cnt = npq;
  a.out_c = b.A;
  a.out_stride = nx;
  a.osc = make_float2(1.f, 0.f);
  a.tag = "phase_fft";
  a.wcnt = b.wcnt;
  a.nwcnt = nwaves;
  a.stats = b.stats;
  a.stats_groups = nparts;
  a.stats_chunks = nchunks;
  a.ready_out = mark ? b.stats + 4 : nullptr;
  a.ready_val = ready_tag(L);
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

static int run_chi_table(const Bufs& b, const float* d_theta, int n_k, const Optics& o, hipStream_t s) {
  STEM_TRACE("chi_table", s);
  hipLaunchKernelGGL(k_chi_table, dim3((n_k + 255) / 256), dim3(256), 0, s, b.kc, d_theta, n_k, o, b.kchi);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

static int run_pair_count(const SsbLayout& L, const Bufs& b, int ny, int nx, hipStream_t s) {
  STEM_TRACE("pair_count", s);
  hipLaunchKernelGGL(k_pair_count, dim3((unsigned)((L.F + 255) / 256)), dim3(256), 0, s, b.cst, L.n_k, ny, nx,
                     b.npq);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

static int run_prune_offsets(const SsbLayout& L, const Bufs& b, int nx, int32_t* d_status, hipStream_t s) {
  STEM_TRACE("prune_offsets", s);
  hipLaunchKernelGGL(k_prune_runs, dim3((unsigned)nx), dim3(256), 0, s, b.cst, L.n_k, nx, b.poff, b.ptot, b.pcs);
  STEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_prune_bases, dim3(1), dim3(256), 0, s, L.n_k, nx, b.poff, b.ptot, L.pcap, d_status);
  STEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_prune_add, dim3((unsigned)nx), dim3(256), 0, s, L.n_k, b.poff, b.ptot);
  STEM_LAUNCH_CHECK();
  // the tables of the refocus sum in balanced pieces (the column costs and spans came with the
  // first pass)
  hipLaunchKernelGGL(k_stream_cands, dim3(kStreamCands), dim3(256), 0, s, nx, (int)L.nws, b.pcs);
  STEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_stream_colseg, dim3(1), dim3(256), 0, s, nx, (int)L.nws, b.pcs);
  STEM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_stream_waves, dim3((unsigned)nx), dim3(256), 0, s, L.n_k, b.poff, nx, b.pcs, b.pws);
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
  return make_layout(*det, *scan, *optics, *ssb, n_k, &L);
}

extern "C" int ssb_state_region(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                                const stem_ssb* ssb, int region, size_t* offset, size_t* bytes) {
  int n_k;
  if (check_common(det, scan, optics, ssb, &n_k) || !offset || !bytes) return STEM_EINVAL;
  SsbLayout L;
  make_layout(*det, *scan, *optics, *ssb, n_k, &L);
  switch (region) {
    case STEM_REGION_D: *offset = L.D; *bytes = (size_t)n_k * L.F * (ssb->d_bits / 8); break;
    case STEM_REGION_X: *offset = L.X; *bytes = (size_t)L.xpix * L.nh * scan->ny * sizeof(float2); break;
    case STEM_REGION_T: *offset = L.T; *bytes = (size_t)L.F * sizeof(float2); break;
    case STEM_REGION_KC: *offset = L.kc; *bytes = (size_t)n_k * sizeof(double2); break;
    case STEM_REGION_STATS: *offset = L.stats; *bytes = 4 * sizeof(unsigned long long); break;
    case STEM_REGION_PG: *offset = L.pg; *bytes = (size_t)L.pcap * sizeof(float2); break;
    case STEM_REGION_POFF:
      *offset = L.poff;
      *bytes = L.store ? sizeof(int64_t) * ((size_t)n_k * scan->nx + 1) : 0;
      break;
    case STEM_REGION_NPAIR: *offset = L.npq; *bytes = (size_t)L.F * sizeof(int32_t); break;
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
  make_layout(*det, *scan, *optics, *ssb, n_k, &L);
  if (!state || ((uintptr_t)state & 255) || state_bytes < L.total) return STEM_EWORKSPACE;
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
    const SetsJob job{o, n_k, nx, ny, L.ncs, L.nmw, b.cst, b.cmask, colset_width(ny)};
    if ((st = launch_bin(d_idx, d_off, frame0, n_frames, *det, o.r2, b.rows, b.kc, b.lut, n_k, L.F, b.D,
                          ssb->d_bits, d_status, s, com, &job, frame0 == 0 ? b.stats + 4 : nullptr)))
      return st;
    if (L.store && L.fast) {
      // STEM_G_STORE keeps the row transform of every pixel: transform this chunk's rows now
      const int ry0 = (int)(frame0 / nx), nr = (int)(n_frames / nx);
      const int64_t nrows = (int64_t)n_k * nr;
      if (ssb->d_bits == 8)
        st = launch_xstage_t<uint8_t>(ssb->precision, nx, (const uint8_t*)b.D, ny, ry0, nr, nrows, b.X, s);
      else
        st = launch_xstage_t<uint16_t>(ssb->precision, nx, (const uint16_t*)b.D, ny, ry0, nr, nrows, b.X, s);
      if (st) return st;
    }
    if (mode == STEM_SSB_ACCUMULATE) return STEM_OK;
  }
  const int chi0 = chi_is_zero(o, d_theta);
  const bool refocus = mode == STEM_SSB_REFOCUS;
  // The interval table and mask depend only on the geometry: ACCUMULATE's binning built them when
  // it bins through its LDS table; otherwise the first sum builds them (a refocus finds them from
  // the FINALIZE before it).  chi(Kc) + theta comes with them, or from its own small kernel.
  // A refocus from the stored values evaluates chi(Kc) + theta per pixel as it gathers the runs.
  if (!refocus && !bin_builds_sets(*det, o.r2)) {
    if ((st = launch_colsets(b.kc, n_k, nx, ny, o, b.cst, b.cmask, L.nmw, s, d_theta, chi0 ? nullptr : b.kchi)))
      return st;
  } else if (!chi0 && !(refocus && L.store)) {
    if ((st = run_chi_table(b, d_theta, n_k, o, s))) return st;
  }
  if (ssb->normalize && !refocus && (st = run_pair_count(L, b, ny, nx, s))) return st;
  YArgs a = yargs(L, b, nx);
  if (refocus) need_finalize(a, L, b, d_status);
  if (L.store && refocus) {
    // Eq. 3 again from the stored double-overlap values
    a.ngroups = L.pgroups;
    a.kch_inline = 1;
    a.theta = d_theta;
    if ((st = launch_psum_stream(ny, a, o, chi0, (int)L.nwq, b.pws, b.pcs, s))) return st;
    return run_phase(L, b, *scan, L.pgroups, L.nwq, 1, ssb->normalize ? b.npq : nullptr, d_phase, d_T, s, false,
                     b.pcs);
  } else if (!L.fast) {
    // the other scan lengths: row and column transforms by the generic FFT, then Eq. 3 per
    // (pixel, column) run over the full columns of G, chunk by chunk
    a.ngroups = L.pgroups;
    if (L.store) {
      if ((st = xstage_generic(L, b, *ssb, ny, nx, 0, n_k, s))) return st;
      if ((st = run_prune_offsets(L, b, nx, d_status, s))) return st;
    }
    for (int ch = 0; ch < L.nchunks; ++ch) {
      int k0, k1;
      chunk_range(L, ch, k0, k1);
      if (L.store) {
        if ((st = colfft_generic(L, ny, k0, k1, b.X + (size_t)k0 * L.nh * ny, b.Y, s))) return st;
        a.X = b.Y;
      } else {
        if ((st = xstage_generic(L, b, *ssb, ny, nx, k0, k1, s))) return st;
        if ((st = colfft_generic(L, ny, k0, k1, b.X, b.X, s))) return st;
      }
      a.xk0 = k0;
      a.k0 = k0;
      a.k1 = k1;
      a.accumulate = ch > 0;
      if ((st = launch_psum(ny, a, o, chi0, L.store, s))) return st;
    }
    return run_phase(L, b, *scan, L.pgroups, L.nwp, L.nchunks, ssb->normalize ? b.npq : nullptr, d_phase, d_T, s,
                     !refocus);
  } else if (L.store) {
    if ((st = run_prune_offsets(L, b, nx, d_status, s))) return st;
    if ((st = launch_yreduce(ssb->precision, ny, a, o, chi0, 1, s))) return st;
  } else {
    // G recomputed chunk by chunk: row transform of the chunk's pixels, then the fused sum on it
    for (int ch = 0; ch < L.nchunks; ++ch) {
      int k0, k1;
      chunk_range(L, ch, k0, k1);
      if ((st = xstage_pixels(L, b, *ssb, ny, nx, k0, k1, s))) return st;
      a.xk0 = k0;
      a.k0 = k0;
      a.k1 = k1;
      a.accumulate = ch > 0;
      if ((st = launch_yreduce(ssb->precision, ny, a, o, chi0, 0, s))) return st;
    }
  }
  return run_phase(L, b, *scan, L.groups, L.nwy, L.store ? 1 : L.nchunks, ssb->normalize ? b.npq : nullptr, d_phase,
                   d_T, s, !refocus);
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
// G(K, Q) at selected Q as binned detector images

struct PanelQ {
  int32_t my[STEM_MAX_PANEL], mx[STEM_MAX_PANEL];
};

// From the row-transformed cube (STEM_G_STORE): one wave per (bin, Q), the DFT along ry of the
// stored column with FP64 accumulation.
__global__ void __launch_bounds__(64) k_g_panel(const float2* __restrict__ X, const RowRun* __restrict__ rows,
                                               int nbx, int n_k, int ny, int nx, PanelQ q, float2* __restrict__ img) {
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
    my = (ny - my) % ny;
  }
  const float2* col = X + ((int64_t)kd * (nx / 2 + 1) + mx) * ny;
  // sum over ry of X exp(-2 pi i my ry / Ny), angles reduced exactly as integers mod Ny
  double re = 0.0, im = 0.0;
  for (int ry = lane; ry < ny; ry += 64) {
    const int k = (int)(((int64_t)my * ry) % ny);
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
  float2 v = make_float2((float)re, (float)im);
  if (cj) v.y = -v.y;
  if (lane == 0) *out = v;
}

// From the binned cube (STEM_G_RECOMPUTE keeps no row-transformed cube): one workgroup per (bin,
// group of kPanelGroup frequencies), the 2D DFT over (ry, rx) at those Q_j with FP64
// accumulation of the rows: each thread sums its columns rx of a row with W_Nx^(mx rx) (held in
// registers for the pass: the same for every row; KC products in FP32), multiplies the row's
// partial by W_Ny^(my ry) in FP64 and adds it;
// twiddles W_N^t for exact integer t (FP64 sincospi rounded to FP32) from LDS, their indices
// advanced by exact integer steps.  The rows' loads are pipelined (kPanelRows in flight), the
// columns taken in passes of kPanelCols.
constexpr int kPanelTw = kGenMax;
#ifndef STEM_PANEL_GROUP
#define STEM_PANEL_GROUP 2
#endif
constexpr int kPanelGroup = STEM_PANEL_GROUP;  // frequencies per workgroup (its unrolled slots)
constexpr int kPanelCols = 1024;  // columns per pass of the workgroup's 256 threads
constexpr int kPanelRows = 8;     // rows of counts in flight

template <typename DT, int GQ>
__global__ void __launch_bounds__(256) k_g_panel_d(const DT* __restrict__ D, const RowRun* __restrict__ rows,
                                                  int nbx, int n_k, int ny, int nx, PanelQ q, int n_q,
                                                  float2* __restrict__ img) {
  __shared__ float2 s_wx[kPanelTw], s_wy[kPanelTw];
  __shared__ double s_red[2][GQ][4];
  const int bin = blockIdx.x;
  const int by = bin / nbx, bx = bin % nbx;
  const int nbins = gridDim.x;
  const int j0 = blockIdx.y * GQ;
  const int nj = min(GQ, n_q - j0);
  const RowRun rr = rows[by];
  const int kd = rr.start + bx - rr.lo;
  if (bx < rr.lo || bx >= rr.hi || kd < 0 || kd >= n_k) {
    for (int j = threadIdx.x; j < nj; j += blockDim.x) img[(int64_t)(j0 + j) * nbins + bin] = make_float2(0.f, 0.f);
    return;
  }
  for (int t = threadIdx.x; t < nx; t += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)t / (double)nx, &sn, &cs);
    s_wx[t] = make_float2((float)cs, (float)-sn);
  }
  for (int t = threadIdx.x; t < ny; t += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)t / (double)ny, &sn, &cs);
    s_wy[t] = make_float2((float)cs, (float)-sn);
  }
  __syncthreads();
  const DT* d = D + (int64_t)kd * ny * nx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // columns in passes of kPanelCols (thread t: rx = cb + t + 256 k, k < kPanelCols / 256); the
  // counts of kPanelRows rows are in flight (rotating register slots, each refilled with the row
  // kPanelRows further on once summed), so the row loop does not wait on every row's loads
  constexpr int KC = kPanelCols / 256, P = kPanelRows;
  int mx[GQ], my[GQ], xs[GQ];
#pragma unroll
  for (int j = 0; j < GQ; ++j) {
    mx[j] = j < nj ? q.mx[j0 + j] : 0;
    my[j] = j < nj ? q.my[j0 + j] : 0;
    xs[j] = (int)(((int64_t)mx[j] * blockDim.x) % nx);  // index step per blockDim.x columns
  }
  double are[GQ], aim[GQ];
#pragma unroll
  for (int j = 0; j < GQ; ++j) are[j] = aim[j] = 0.0;
  for (int cb = 0; cb < nx; cb += kPanelCols) {
    // the x twiddles of this thread's columns are the same for every row of the pass
    float twr[GQ][KC], twi[GQ][KC];
    int yi[GQ];
#pragma unroll
    for (int j = 0; j < GQ; ++j) {
      int xi = (int)(((int64_t)mx[j] * (cb + (int)threadIdx.x)) % nx);  // this thread's first rx
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const float2 w = s_wx[xi];
        twr[j][k] = w.x;
        twi[j][k] = w.y;
        xi += xs[j];
        if (xi >= nx) xi -= nx;
      }
      yi[j] = 0;  // my ry mod Ny
    }
    uint32_t cnt[P][KC];
    // every load is issued (past the last row or column it reads an in-range count, dropped where
    // the count is used), so the wait counts of the pipelined loop stay exact
    bool colok[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) colok[k] = cb + (int)threadIdx.x + 256 * k < nx;
    auto load_row = [&](int ry, uint32_t* dst) {
      const int64_t row = (int64_t)min(ry, ny - 1) * nx;
#pragma unroll
      for (int k = 0; k < KC; ++k) dst[k] = (uint32_t)d[row + min(cb + (int)threadIdx.x + 256 * k, nx - 1)];
    };
#pragma unroll
    for (int p = 0; p < P; ++p) load_row(p, cnt[p]);
    for (int ry0 = 0; ry0 < ny; ry0 += P) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int ry = ry0 + p;
        const bool rowok = ry < ny;  // past the last row: counts dropped, the row adds 0
        // the thread's partial of the row: KC products in FP32 (counts below 2^16 are exact; at
        // Q = 0 every product and sum is an exact integer), then FP64
        float fre[GQ], fim[GQ];
#pragma unroll
        for (int j = 0; j < GQ; ++j) fre[j] = fim[j] = 0.f;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
          const float c = (float)(rowok && colok[k] ? cnt[p][k] : 0u);
#pragma unroll
          for (int j = 0; j < GQ; ++j) {
            fre[j] = fmaf(c, twr[j][k], fre[j]);
            fim[j] = fmaf(c, twi[j][k], fim[j]);
          }
        }
        double rre[GQ], rim[GQ];
#pragma unroll
        for (int j = 0; j < GQ; ++j) {
          rre[j] = (double)fre[j];
          rim[j] = (double)fim[j];
        }
        load_row(ry + P, cnt[p]);
#pragma unroll
        for (int j = 0; j < GQ; ++j) {
          const float2 w = s_wy[yi[j]];
          are[j] += rre[j] * (double)w.x - rim[j] * (double)w.y;
          aim[j] += rre[j] * (double)w.y + rim[j] * (double)w.x;
          yi[j] += my[j];
          if (yi[j] >= ny) yi[j] -= ny;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < GQ; ++j) {
    double re = are[j], im = aim[j];
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) {
      s_red[0][j][wave] = re;
      s_red[1][j][wave] = im;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nj) {
    const int j = threadIdx.x;
    const double tr = (s_red[0][j][0] + s_red[0][j][1]) + (s_red[0][j][2] + s_red[0][j][3]);
    const double ti = (s_red[1][j][0] + s_red[1][j][1]) + (s_red[1][j][2] + s_red[1][j][3]);
    img[(int64_t)(j0 + j) * nbins + bin] = make_float2((float)tr, (float)ti);
  }
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
  make_layout(*det, *scan, *optics, *ssb, n_k, &L);
  if (!state || ((uintptr_t)state & 255) || state_bytes < L.total) return STEM_EWORKSPACE;
  const Bufs b = carve(const_cast<void*>(state), L);
  const int nbx = det->W / det->bin, nby = det->H / det->bin;
  hipStream_t s = (hipStream_t)stream_;
  STEM_TRACE("g_panel", s);
  if (L.store) {
    hipLaunchKernelGGL(k_g_panel, dim3((unsigned)(nbx * nby), (unsigned)n_q), dim3(64), 0, s, b.X, b.rows, nbx, n_k,
                       scan->ny, scan->nx, q, (float2*)d_img);
  } else if (scan->nx > kPanelTw || scan->ny > kPanelTw) {
    return STEM_EINVAL;
  } else {
    const dim3 grid((unsigned)(nbx * nby), (unsigned)((n_q + kPanelGroup - 1) / kPanelGroup));
    if (ssb->d_bits == 8)
      hipLaunchKernelGGL((k_g_panel_d<uint8_t, kPanelGroup>), grid, dim3(256), 0, s, (const uint8_t*)b.D, b.rows, nbx, n_k,
                         scan->ny, scan->nx, q, n_q, (float2*)d_img);
    else
      hipLaunchKernelGGL((k_g_panel_d<uint16_t, kPanelGroup>), grid, dim3(256), 0, s, (const uint16_t*)b.D, b.rows, nbx, n_k,
                         scan->ny, scan->nx, q, n_q, (float2*)d_img);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

extern "C" int ssb_backward(const float* d_dLdphi, const stem_det* det, const stem_scan* scan,
                            const stem_optics* optics, const stem_ssb* ssb, const float* d_theta, void* state,
                            size_t state_bytes, double* d_dLdc, float* d_dLdtheta, int32_t* d_status,
                            void* stream_) {
  int n_k;
  int st = check_common(det, scan, optics, ssb, &n_k);
  if (st) return st;
  if (!d_dLdphi || !d_dLdc || ssb->normalize) return STEM_EINVAL;
  SsbLayout L;
  make_layout(*det, *scan, *optics, *ssb, n_k, &L);
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
  // chi(Kc) + theta for these coefficients (evaluated per pixel by the adjoint over the stored
  // values); the interval table and mask are the last sum's
  if (!L.store && (st = run_chi_table(b, d_theta, n_k, o, s))) return st;
  YArgs y = yargs(L, b, nx);
  need_finalize(y, L, b, d_status);
  int64_t npdc = L.nwy, npdth = L.ncs;
  const int64_t* pieces = nullptr;
  if (L.store) {
    y.kch_inline = 1;
    y.theta = d_theta;
    if ((st = launch_padj_stream(ny, y, o, (int)L.nwq, b.pws, b.pcs, s))) return st;
    npdc = L.nwq;
    npdth = nx;
    pieces = b.pcs;
  } else if (!L.fast) {
    y.ngroups = L.pgroups;
    for (int ch = 0; ch < L.nchunks; ++ch) {
      int k0, k1;
      chunk_range(L, ch, k0, k1);
      if ((st = xstage_generic(L, b, *ssb, ny, nx, k0, k1, s))) return st;
      if ((st = colfft_generic(L, ny, k0, k1, b.X, b.X, s))) return st;
      y.xk0 = k0;
      y.k0 = k0;
      y.k1 = k1;
      y.accumulate = ch > 0;
      if ((st = launch_padj(ny, y, o, s))) return st;
    }
    npdc = L.nwa;
    npdth = nx;
  } else {
    for (int ch = 0; ch < L.nchunks; ++ch) {
      int k0, k1;
      chunk_range(L, ch, k0, k1);
      if ((st = xstage_pixels(L, b, *ssb, ny, nx, k0, k1, s))) return st;
      y.xk0 = k0;
      y.k0 = k0;
      y.k1 = k1;
      y.accumulate = ch > 0;
      if ((st = launch_yadjoint(ssb->precision, ny, y, o, s))) return st;
    }
  }
  {
    STEM_TRACE("ssb_adjoint_final", s);
    hipLaunchKernelGGL(k_adjoint_final, dim3(kFinalDcBlocks + (n_k + 3) / 4), dim3(256), 0, s, b.pdc, npdc, b.pdth,
                       npdth, n_k, pieces, d_dLdc, d_dLdtheta);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
