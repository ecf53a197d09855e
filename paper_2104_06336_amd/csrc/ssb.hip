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
#include "kernels.h"
#include "optics.h"
#include "trace.h"

namespace stem {

constexpr int kXThreads = 512;
constexpr int kXWaveStride = kFftLds + 4;
constexpr int kMaxPixels = 4096;

struct SsbLayout {
  int n_k, nby, nh;
  int64_t F;
  size_t rows, kc, kchi, stats, D, X, T, A, Tb, pdc, pdth, total;
  int64_t nblk;  // workgroups of the per-Q kernels
};

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
  L->stats = o; o = align256(o + sizeof(unsigned long long) * 4);
  L->D = o;     o = align256(o + (size_t)n_k * L->F * (ssb.d_bits / 8));
  L->X = o;     o = align256(o + (size_t)n_k * L->nh * scan.ny * sizeof(float2));
  L->T = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->A = o;     o = align256(o + (size_t)L->F * sizeof(float2));
  L->Tb = o;    o = align256(o + (size_t)L->F * sizeof(float2));
  L->pdc = o;   o = align256(o + (size_t)L->nblk * 8 * sizeof(double));
  L->pdth = o;  o = align256(o + (size_t)L->nblk * 4 * n_k * sizeof(float));
  L->total = o;
  return o;
}

// ---------------------------------------------------------------------------------------------
// x-stage: rows (kd, ry) with ry in [ry0, ry0 + nr) of D, two real rows per complex FFT.
// Tile = 16B real rows (B = 1024/N); each of the 8 waves transforms B row pairs; the
// workgroup then splits the pairs and writes X[kd][m][ry] for m in [0, N/2] in runs of
// consecutive ry.

template <int N, typename DT>
__global__ void __launch_bounds__(kXThreads) k_xstage(const DT* __restrict__ D, int ny, int ry0, int nr,
                                                      int64_t nrows, float2* __restrict__ X) {
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[8 * kXWaveStride];
  constexpr int B = 1024 / N;
  constexpr int TR = 16 * B;
  constexpr int NH = N / 2 + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  fill_twiddles(s_tw, threadIdx.x, kXThreads);
  __syncthreads();
  float2* buf = s_buf + wave * kXWaveStride;
  const int64_t ntiles = (nrows + TR - 1) / TR;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TR + wave * 2 * B;
    float2 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, n;
      fft_in_index<N>(lane, i, b, n);
      const int64_t ra = r0 + 2 * b;
      float re = 0.f, im = 0.f;
      if (ra < nrows) {
        const int64_t kd = ra / nr, ry = ry0 + ra % nr;
        re = (float)D[(kd * ny + ry) * N + n];
      }
      if (ra + 1 < nrows) {
        const int64_t kd = (ra + 1) / nr, ry = ry0 + (ra + 1) % nr;
        im = (float)D[(kd * ny + ry) * N + n];
      }
      v[i] = make_float2(re, im);
    }
    wave_fft<N>(v, buf, s_tw, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      fft_out_index<N>(lane, i, b, m);
      buf[fft_pad(b * N + m)] = v[i];
    }
    __syncthreads();
    for (int u = threadIdx.x; u < NH * TR; u += kXThreads) {
      const int m = u / TR, rl = u % TR;
      const int w = rl / (2 * B), p = rl % (2 * B);
      const int b = p >> 1;
      const float2* wb = s_buf + w * kXWaveStride;
      const float2 z = wb[fft_pad(b * N + m)];
      const float2 zc = cconj(wb[fft_pad(b * N + ((N - m) & (N - 1)))]);
      // row 2b: (z + conj z(-m))/2 ; row 2b+1: (z - conj z(-m))/(2i)
      const float2 val = (p & 1) ? cscale(cmul_mi(csub(z, zc)), 0.5f) : cscale(cadd(z, zc), 0.5f);
      const int64_t rho = tile * TR + rl;
      if (rho < nrows) {
        const int64_t kd = rho / nr, ry = ry0 + rho % nr;
        X[(kd * NH + m) * ny + ry] = val;
      }
    }
    __syncthreads();
  }
}

template <typename DT>
static int launch_xstage_t(int nx, const DT* D, int ny, int ry0, int nr, int64_t nrows, float2* X,
                           hipStream_t s) {
  const int64_t tr = 16 * (1024 / nx);
  const int64_t tiles = (nrows + tr - 1) / tr;
  const dim3 grid((unsigned)(tiles < 4096 ? tiles : 4096)), blk(kXThreads);
  STEM_TRACE("xstage_fft", s);
  switch (nx) {
    case 32: hipLaunchKernelGGL((k_xstage<32, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    case 64: hipLaunchKernelGGL((k_xstage<64, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    case 128: hipLaunchKernelGGL((k_xstage<128, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    case 256: hipLaunchKernelGGL((k_xstage<256, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    case 512: hipLaunchKernelGGL((k_xstage<512, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    case 1024: hipLaunchKernelGGL((k_xstage<1024, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, X); break;
    default: return STEM_EINVAL;
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// chi(Kc) + theta per kept pixel

__global__ void k_chi_table(const double2* __restrict__ kc, const float* __restrict__ theta, int n_k,
                            Optics o, double* __restrict__ kchi, unsigned long long* __restrict__ stats) {
  const int kd = blockIdx.x * blockDim.x + threadIdx.x;
  if (kd < 4) stats[kd] = 0ull;  // counters of the sum that follows
  if (kd >= n_k) return;
  const double2 k = kc[kd];
  kchi[kd] = chi_px(k.x, k.y, o) + (theta ? (double)theta[kd] : 0.0);
}

// ---------------------------------------------------------------------------------------------
// Eq. 3 from a stored G: one thread per Q, Q in column-major order q = mx*Ny + my.

__global__ void __launch_bounds__(256) k_reduce(const float2* __restrict__ G, const double2* __restrict__ kc,
                                                const double* __restrict__ kchi, int n_k, int ny, int nx,
                                                Optics o, int normalize, float2* __restrict__ Tt,
                                                unsigned long long* __restrict__ stats) {
  const int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q0 < (int64_t)ny * nx;
  const int64_t q = valid ? q0 : 0;
  const int mx = (int)(q / ny), my = (int)(q % ny);
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const double qy = (double)signed_index(my, ny) * o.sy;
  const bool mir = mx > nx / 2;
  const int gmx = mir ? nx - mx : mx, gmy = mir ? (ny - my) % ny : my;
  const int nh = nx / 2 + 1;
  const float2* gcol = G + (int64_t)gmx * ny + gmy;
  const int64_t kstride = (int64_t)nh * ny;
  float2 acc = make_float2(0.f, 0.f);
  int cnt = 0;
  for (int kd = 0; kd < n_k && valid; ++kd) {
    const double2 k = kc[kd];
    if (!double_overlap(k.x, k.y, qx, qy, o.r2)) continue;
    const double psi = chi_px(k.x - qx, k.y - qy, o) - kchi[kd];
    float2 g = gcol[kd * kstride];
    if (mir) g = cconj(g);
    const float2 e = expi_reduced(psi);
    acc.x += g.x * e.x - g.y * e.y;
    acc.y += g.x * e.y + g.y * e.x;
    ++cnt;
  }
  if (normalize && cnt > 0) acc = cscale(acc, 1.f / (float)cnt);
  if (valid) Tt[q] = acc;
  // number of double-overlap pairs of this sum, one atomic per wave
  unsigned long long c = valid ? (unsigned long long)cnt : 0ull;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(stats, c);
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
// adjoint from a stored G, one thread per Q (same traversal as k_reduce).
//   w = Re(conj(Tbar) i G e^{i psi});  dc_j += w (B_j(K - Q) - B_j(K));  dtheta[kd] -= w

__global__ void __launch_bounds__(256) k_adjoint(const float2* __restrict__ G, const double2* __restrict__ kc,
                                                 const double* __restrict__ kchi, int n_k, int ny, int nx,
                                                 Optics o, const float2* __restrict__ Tbt,
                                                 double* __restrict__ pdc, float* __restrict__ pdth) {
  __shared__ double s_dc[4][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < (int64_t)ny * nx;
  const int mx = valid ? (int)(q / ny) : 0, my = valid ? (int)(q % ny) : 0;
  const double qx = (double)signed_index(mx, nx) * o.sx;
  const double qy = (double)signed_index(my, ny) * o.sy;
  const bool mir = mx > nx / 2;
  const int gmx = mir ? nx - mx : mx, gmy = mir ? (ny - my) % ny : my;
  const int nh = nx / 2 + 1;
  const float2* gcol = G + (int64_t)gmx * ny + gmy;
  const int64_t kstride = (int64_t)nh * ny;
  const float2 tb = valid ? Tbt[q] : make_float2(0.f, 0.f);
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  for (int kd = 0; kd < n_k; ++kd) {
    const double2 k = kc[kd];
    const bool in = valid && double_overlap(k.x, k.y, qx, qy, o.r2);
    float w = 0.f;
    if (in) {
      double bm[8], bk[8];
      chi_basis(k.x - qx, k.y - qy, o, bm);
      double chim = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j) chim += o.c[j] * bm[j];
      const double psi = chim - kchi[kd];
      float2 g = gcol[kd * kstride];
      if (mir) g = cconj(g);
      const float2 e = expi_reduced(psi);
      const float2 z = make_float2(g.x * e.x - g.y * e.y, g.x * e.y + g.y * e.x);
      // Re(conj(tb) * (i z)) with i z = (-z.y, z.x)
      w = tb.x * (-z.y) + tb.y * z.x;
      chi_basis(k.x, k.y, o, bk);
#pragma unroll
      for (int j = 0; j < 8; ++j) dc[j] += (double)w * (bm[j] - bk[j]);
    }
    // per-wave sum for dtheta[kd] in a fixed butterfly order, one partial per wave
    float sw = 0.f;
    if (__ballot(in) != 0) {
      sw = w;
      for (int off = 32; off > 0; off >>= 1) sw += __shfl_xor(sw, off);
    }
    if (lane == 0) pdth[((int64_t)blockIdx.x * 4 + wave) * n_k + kd] = -sw;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double s = dc[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) s_dc[wave][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < 8)
    pdc[blockIdx.x * 8 + threadIdx.x] =
        ((s_dc[0][threadIdx.x] + s_dc[1][threadIdx.x]) + s_dc[2][threadIdx.x]) + s_dc[3][threadIdx.x];
}

// sums the per-workgroup partials in a fixed order
__global__ void __launch_bounds__(256) k_adjoint_final(const double* __restrict__ pdc, const float* __restrict__ pdth,
                                                       int64_t nblk, int n_k, double* __restrict__ dLdc,
                                                       float* __restrict__ dLdth) {
  __shared__ double s[256][8];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x)
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
  if (dLdth)
    for (int kd = threadIdx.x; kd < n_k; kd += blockDim.x) {
      double a = 0.0;
      for (int64_t b = 0; b < 4 * nblk; ++b) a += (double)pdth[b * n_k + kd];
      dLdth[kd] = (float)a;
    }
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
  return o;
}

struct Bufs {
  RowRun* rows;
  double2* kc;
  double* kchi;
  unsigned long long* stats;
  void* D;
  float2* X;
  float2* T;
  float2* A;
  float2* Tb;
  double* pdc;
  float* pdth;
};

static Bufs carve(void* state, const SsbLayout& L) {
  char* p = (char*)state;
  return Bufs{(RowRun*)(p + L.rows), (double2*)(p + L.kc), (double*)(p + L.kchi),
              (unsigned long long*)(p + L.stats), (void*)(p + L.D),
              (float2*)(p + L.X),    (float2*)(p + L.T),  (float2*)(p + L.A),     (float2*)(p + L.Tb),
              (double*)(p + L.pdc),  (float*)(p + L.pdth)};
}

static int check_common(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                        const stem_ssb* ssb, int* n_k) {
  if (!det_ok(det) || !scan || !optics_ok(optics) || !ssb) return STEM_EINVAL;
  if (!is_pow2_in(scan->ny, 32, 1024) || !is_pow2_in(scan->nx, 32, 1024) || !(scan->step > 0))
    return STEM_EINVAL;
  if (ssb->d_bits != 8 && ssb->d_bits != 16) return STEM_EINVAL;
  if (ssb->precision != STEM_FFT_FP32) return STEM_EINVAL;
  if (ssb->g_mode != STEM_G_STORE && ssb->g_mode != STEM_G_RECOMPUTE) return STEM_EINVAL;
  const int n = count_pixels(*det, optics->r_bf * optics->r_bf);
  if (n <= 0 || n > kMaxPixels) return STEM_EINVAL;
  *n_k = n;
  return STEM_OK;
}

static int run_phase(const SsbLayout& L, const Bufs& b, const stem_scan& sc, float* d_phase, float* d_T,
                     hipStream_t s) {
  const int ny = sc.ny, nx = sc.nx;
  if (d_phase) {
    RowFftArgs a{};
    // inverse along my of each mx row of T -> A[ry][mx]
    a.nrows = nx;
    a.in_c = b.T;
    a.nparts = 1;
    a.part_stride = 0;
    a.out_c = b.A;
    a.out_stride = nx;
    a.osc = make_float2(1.f, 0.f);
    a.tag = "phase_fft";
    int st = launch_row_fft(ny, true, IN_C64_SUM, OUT_T_C64, a, s);
    if (st) return st;
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

extern "C" int ssb_reconstruct(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                               const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                               const stem_ssb* ssb, int mode, const float* d_theta, void* state,
                               size_t state_bytes, float* d_phase, float* d_T, int32_t* d_status,
                               void* stream_) {
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
    if ((st = launch_geometry(*det, o.r2, b.rows, b.kc, s))) return st;
    if ((st = launch_bin(d_idx, d_off, frame0, n_frames, *det, b.rows, n_k, L.F, b.D, ssb->d_bits, d_status, s)))
      return st;
    const int ry0 = (int)(frame0 / nx), nr = (int)(n_frames / nx);
    const int64_t nrows = (int64_t)n_k * nr;
    if (ssb->d_bits == 8)
      st = launch_xstage_t<uint8_t>(nx, (const uint8_t*)b.D, ny, ry0, nr, nrows, b.X, s);
    else
      st = launch_xstage_t<uint16_t>(nx, (const uint16_t*)b.D, ny, ry0, nr, nrows, b.X, s);
    if (st) return st;
    if (mode == STEM_SSB_ACCUMULATE) return STEM_OK;
  }
  if (mode == STEM_SSB_FINALIZE || mode == STEM_SSB_ONESHOT) {
    // column transform along ry, in place: X -> G
    RowFftArgs a{};
    a.nrows = (int64_t)n_k * L.nh;
    a.in_c = b.X;
    a.out_c = b.X;
    a.osc = make_float2(1.f, 0.f);
    a.tag = "ystage_fft";
    if ((st = launch_row_fft(ny, false, IN_C64, OUT_ROW_C64, a, s))) return st;
  }
  {
    STEM_TRACE("chi_table", s);
    hipLaunchKernelGGL(k_chi_table, dim3((n_k + 255) / 256), dim3(256), 0, s, b.kc, d_theta, n_k, o, b.kchi, b.stats);
  }
  STEM_LAUNCH_CHECK();
  {
    STEM_TRACE("ssb_reduce", s);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)L.nblk), dim3(256), 0, s, b.X, b.kc, b.kchi, n_k, ny, nx, o,
                       ssb->normalize, b.T, b.stats);
  }
  STEM_LAUNCH_CHECK();
  return run_phase(L, b, *scan, d_phase, d_T, s);
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
  {
    STEM_TRACE("chi_table", s);
    hipLaunchKernelGGL(k_chi_table, dim3((n_k + 255) / 256), dim3(256), 0, s, b.kc, d_theta, n_k, o, b.kchi, b.stats);
  }
  STEM_LAUNCH_CHECK();
  {
    STEM_TRACE("ssb_adjoint", s);
    hipLaunchKernelGGL(k_adjoint, dim3((unsigned)L.nblk), dim3(256), 0, s, b.X, b.kc, b.kchi, n_k, ny, nx, o,
                       b.Tb, b.pdc, b.pdth);
  }
  STEM_LAUNCH_CHECK();
  {
    STEM_TRACE("ssb_adjoint_final", s);
    hipLaunchKernelGGL(k_adjoint_final, dim3(1), dim3(256), 0, s, b.pdc, b.pdth, L.nblk, n_k, d_dLdc,
                       d_dLdtheta);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
