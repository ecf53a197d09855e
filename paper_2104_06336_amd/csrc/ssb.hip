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
  size_t rows, kc, kchi, stats, D, X, T, A, Tb, pdc, pdth, part, total;
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
                                                      int64_t nrows, int pair_store, float2* __restrict__ X) {
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[8 * kXWaveStride];
  constexpr int B = 1024 / N;
  constexpr int TR = 16 * B;  // real rows per tile
  constexpr int NH = N / 2 + 1;
  constexpr int ROWB = N * (int)sizeof(DT);  // bytes per row of D
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  fill_twiddles(s_tw, threadIdx.x, kXThreads);
  __syncthreads();
  float2* buf = s_buf + wave * kXWaveStride;
  const int64_t ntiles = (nrows + TR - 1) / TR;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TR + wave * 2 * B;  // first real row of this wave
    // stage the wave's 2B rows of D in its LDS buffer with 16-byte loads
    {
      uint4* raw = (uint4*)buf;
      constexpr int CH = 2 * B * ROWB / 16;  // 16-byte chunks
#pragma unroll
      for (int c = lane; c < CH; c += kWave) {
        const int j = c * 16 / ROWB, col = c * 16 % ROWB;
        const int64_t r = r0 + j;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r < nrows) {
          const int64_t kd = r / nr, ry = ry0 + r % nr;
          v = *(const uint4*)((const char*)D + (kd * ny + ry) * ROWB + col);
        }
        raw[c] = v;
      }
    }
    wave_lds_sync();
    float2 v[16];
    {
      const DT* rows = (const DT*)buf;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        fft_in_index<N>(lane, i, b, n);
        v[i] = make_float2((float)rows[(2 * b) * N + n], (float)rows[(2 * b + 1) * N + n]);
      }
    }
    wave_lds_sync();
    wave_fft<N>(v, buf, s_tw, lane);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      fft_out_index<N>(lane, i, b, m);
      buf[fft_pad(b * N + m)] = v[i];
    }
    __syncthreads();
    // split each complex transform z = a + i b of rows (2p, 2p+1) into the two half spectra
    // A(m) = (z(m) + conj z(-m))/2, B(m) = (z(m) - conj z(-m))/(2i); write them at adjacent ry
    for (int u = threadIdx.x; u < NH * (TR / 2); u += kXThreads) {
      const int m = u / (TR / 2), pr = u % (TR / 2);
      const int w = pr / B, b = pr % B;
      const float2* wb = s_buf + w * kXWaveStride;
      const float2 z = wb[fft_pad(b * N + m)];
      const float2 zc = cconj(wb[fft_pad(b * N + ((N - m) & (N - 1)))]);
      const float2 va = cscale(cadd(z, zc), 0.5f);
      const float2 vb = cscale(cmul_mi(csub(z, zc)), 0.5f);
      const int64_t rho = tile * TR + 2 * pr;
      if (pair_store && rho + 1 < nrows) {
        const int64_t kd = rho / nr, ry = ry0 + rho % nr;
        *(float4*)(X + (kd * NH + m) * ny + ry) = make_float4(va.x, va.y, vb.x, vb.y);
      } else {
        if (rho < nrows) {
          const int64_t kd = rho / nr, ry = ry0 + rho % nr;
          X[(kd * NH + m) * ny + ry] = va;
        }
        if (rho + 1 < nrows) {
          const int64_t kd = (rho + 1) / nr, ry = ry0 + (rho + 1) % nr;
          X[(kd * NH + m) * ny + ry] = vb;
        }
      }
    }
    __syncthreads();
  }
}

template <typename DT>
static int launch_xstage_t(int nx, const DT* D, int ny, int ry0, int nr, int64_t nrows, float2* X,
                           hipStream_t s) {
  const int64_t tr = 16 * (1024 / nx);
  // rows 2p, 2p+1 of a tile share a pixel and sit at adjacent, 16-byte aligned ry when the
  // chunk starts on an even row and holds an even number of rows per pixel
  const int pair_store = (nr % 2 == 0) && (ry0 % 2 == 0);
  const int64_t tiles = (nrows + tr - 1) / tr;
  const dim3 grid((unsigned)(tiles < 4096 ? tiles : 4096)), blk(kXThreads);
  STEM_TRACE("xstage_fft", s);
  switch (nx) {
    case 32: hipLaunchKernelGGL((k_xstage<32, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    case 64: hipLaunchKernelGGL((k_xstage<64, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    case 128: hipLaunchKernelGGL((k_xstage<128, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    case 256: hipLaunchKernelGGL((k_xstage<256, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    case 512: hipLaunchKernelGGL((k_xstage<512, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    case 1024: hipLaunchKernelGGL((k_xstage<1024, DT>), grid, blk, 0, s, D, ny, ry0, nr, nrows, pair_store, X); break;
    default: return STEM_EINVAL;
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
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

// ---------------------------------------------------------------------------------------------
// Fused column transform + Eq. 3 (the path that never stores G).  A wave owns B = 1024/NY
// consecutive half-spectrum columns c (Qx = c*sx) and a group of kept pixels.  For each pixel it
// loads the row-transformed columns X[kd][c][0..NY), FFTs them along ry in registers (giving
// G(kd, (my, c)) for every my), and adds every double-overlap term to its accumulators: the
// direct frequency Q = (my, c) with G, and for 0 < c < Nx/2 the mirrored frequency
// (-my, -c) with conj G.  A pixel is skipped without loading when neither Qx nor -Qx of any of
// its columns lies within r of Kx (then |Kx - Qx| >= r rules out |K - Q| < r for every my).
// The wave writes its partial T for its columns into part[g] (column-major [mx][my]); the phase
// pass sums the groups in a fixed order.  With store_g the transformed columns are also written
// back in place (X becomes G) for later refocusing.

constexpr int kYThreads = 256;

// Registers of a lane grouped by column: register i holds the frequency (my, c0 + b) of
// fft_out_index.  With NB = NY/RL >= 64 the column of register i does not depend on the lane
// (slot = that column offset b); otherwise a slot is the group i/RL, whose column depends on the
// lane.  Per slot the double-overlap sets of the column (and of its mirror) are computed once.
template <int NY>
struct Slots {
  static constexpr int RL = fft_last_radix<NY>();
  static constexpr int NB = NY / RL;
  static constexpr bool uniform_col = NB >= kWave;
  static constexpr int slot_of(int i) { return uniform_col ? (kWave * (i / RL)) / NB : i / RL; }
  static constexpr int count = slot_of(15) + 1;
};

// Double-overlap sets of pixel K along column ix: iy in [a0, a1] but not in [b0, b1].
struct ColSet {
  int a0, a1, b0, b1;
  __device__ __forceinline__ bool has(int iy) const { return iy >= a0 && iy <= a1 && !(iy >= b0 && iy <= b1); }
  __device__ __forceinline__ bool empty() const { return a0 > a1; }
};

__device__ __forceinline__ ColSet col_set(double kx, double ky, int ix, int ny, const Optics& o) {
  const double qx = (double)ix * o.sx;
  ColSet cs;
  disk_interval(kx, ky, qx, o.sy, o.r, o.r2, -1, ny, cs.a0, cs.a1);
  if (cs.a0 > cs.a1) {
    cs.b0 = 1;
    cs.b1 = 0;
    return cs;
  }
  disk_interval(kx, ky, qx, o.sy, o.r, o.r2, +1, ny, cs.b0, cs.b1);
  return cs;
}

template <int NY>
__global__ void __launch_bounds__(kYThreads) k_yreduce(float2* __restrict__ X, const double2* __restrict__ kc,
                                                       const double* __restrict__ kchi, int n_k, int nx,
                                                       int ngroups, Optics o, int store_g,
                                                       float2* __restrict__ part,
                                                       unsigned long long* __restrict__ stats) {
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[4 * kXWaveStride];
  constexpr int B = 1024 / NY;
  using SL = Slots<NY>;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nc = nx / 2 + 1;
  const int ncs = (nc + B - 1) / B;                       // column sets
  const int g = blockIdx.x % ngroups;
  const int cs = (blockIdx.x / ngroups) * 4 + wave;       // this wave's column set
  fill_twiddles(s_tw, threadIdx.x, kYThreads);
  __syncthreads();
  if (cs >= ncs) return;
  float2* buf = s_buf + wave * kXWaveStride;
  const int c0 = cs * B;
  const int kd_a = (int)((int64_t)n_k * g / ngroups), kd_b = (int)((int64_t)n_k * (g + 1) / ngroups);
  float2 accd[16], accm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) accd[i] = accm[i] = make_float2(0.f, 0.f);
  unsigned cnt = 0;
  const int64_t kstride = (int64_t)nc * NY;
  for (int kd = kd_a; kd < kd_b; ++kd) {
    const double2 k = kc[kd];
    // double-overlap sets of this pixel for the lane's columns (direct and mirrored)
    ColSet sd[SL::count], sm[SL::count];
    bool any = false;
#pragma unroll
    for (int sl = 0; sl < SL::count; ++sl) {
      int b0, m0;
      fft_out_index<NY>(lane, sl * (16 / SL::count), b0, m0);
      int c = c0 + b0;
      asm volatile("" : "+v"(c));
      sd[sl] = ColSet{1, 0, 1, 0};
      sm[sl] = ColSet{1, 0, 1, 0};
      if (c < nc) {
        sd[sl] = col_set(k.x, k.y, signed_index(c, nx), NY, o);
        if (c > 0 && 2 * c < nx) sm[sl] = col_set(k.x, k.y, signed_index(nx - c, nx), NY, o);
      }
      any = any || !sd[sl].empty() || !sm[sl].empty();
    }
    // with store_g every pixel is transformed, so that the stored G is complete
    if (!store_g && !__ballot(any)) continue;
    float2 v[16];
    const float2* xcol = X + kd * kstride + (int64_t)c0 * NY;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, n;
      fft_in_index<NY>(lane, i, b, n);
      v[i] = (c0 + b < nc) ? xcol[(int64_t)b * NY + n] : make_float2(0.f, 0.f);
    }
    wave_fft<NY>(v, buf, s_tw, lane);
    if (store_g) {
      float2* gcol = X + kd * kstride + (int64_t)c0 * NY;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, m;
        fft_out_index<NY>(lane, i, b, m);
        if (c0 + b < nc) gcol[(int64_t)b * NY + m] = v[i];
      }
    }
    const double kch = kchi[kd];
#pragma unroll
    for (int sl = 0; sl < SL::count; ++sl) {
      int b0, m0;
      fft_out_index<NY>(lane, sl * (16 / SL::count), b0, m0);
      const int c = c0 + b0;
      const ChiCol chd = chi_column(o.lk * (k.x - (double)signed_index(c, nx) * o.sx), o);
      const ChiCol chm = chi_column(o.lk * (k.x - (double)signed_index(nx - c, nx) * o.sx), o);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (SL::slot_of(i) != sl) continue;
        int b, m;
        fft_out_index<NY>(lane, i, b, m);
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
  float2* pg = part + (int64_t)g * nx * NY;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int b, m;
    fft_out_index<NY>(lane, i, b, m);
    const int c = c0 + b;
    if (c >= nc) continue;
    pg[(int64_t)c * NY + m] = accd[i];
    if (c > 0 && 2 * c < nx) pg[(int64_t)(nx - c) * NY + ((NY - m) & (NY - 1))] = accm[i];
  }
  unsigned long long cc = cnt;
  for (int off = 32; off > 0; off >>= 1) cc += __shfl_xor(cc, off);
  if (lane == 0) atomicAdd(stats, cc);
}

// Fused column transform + adjoint of Eq. 3 (G recomputed, never stored).  Same work split as
// k_yreduce.  For every double-overlap pair, z = G e^{i psi} (conj G for mirrored frequencies),
// w = Re(conj(Tbar(Q)) i z); dL/dc_j gains w (B_j(K - Q) - B_j(K)) and dL/dtheta[kd] loses w.
// Partials: pdc[wave][8] (FP64), pdth[column set][kd] (FP32; one writer per entry).
template <int NY>
__global__ void __launch_bounds__(kYThreads) k_yadjoint(const float2* __restrict__ X, const double2* __restrict__ kc,
                                                        const double* __restrict__ kchi, int n_k, int nx,
                                                        int ngroups, Optics o, int g_stored,
                                                        const float2* __restrict__ Tbt, double* __restrict__ pdc,
                                                        float* __restrict__ pdth) {
  __shared__ float2 s_tw[1024];
  __shared__ float2 s_buf[4 * kXWaveStride];
  constexpr int B = 1024 / NY;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nc = nx / 2 + 1;
  const int ncs = (nc + B - 1) / B;
  const int g = blockIdx.x % ngroups;
  const int cs = (blockIdx.x / ngroups) * 4 + wave;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  fill_twiddles(s_tw, threadIdx.x, kYThreads);
  __syncthreads();
  if (cs >= ncs) {
    if (lane < 8) pdc[wid * 8 + lane] = 0.0;
    return;
  }
  float2* buf = s_buf + wave * kXWaveStride;
  const int c0 = cs * B;
  const int kd_a = (int)((int64_t)n_k * g / ngroups), kd_b = (int)((int64_t)n_k * (g + 1) / ngroups);
  const int ct = c0 + lane % B;
  const bool ct_ok = ct < nc;
  const double ctx = (double)signed_index(ct, nx) * o.sx;
  const bool ct_m = ct_ok && ct > 0 && 2 * ct < nx;
  float2 tbd[16], tbm[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int b, m;
    fft_out_index<NY>(lane, i, b, m);
    const int c = c0 + b;
    tbd[i] = c < nc ? Tbt[(int64_t)c * NY + m] : make_float2(0.f, 0.f);
    tbm[i] = (c < nc && c > 0 && 2 * c < nx) ? Tbt[(int64_t)(nx - c) * NY + ((NY - m) & (NY - 1))]
                                              : make_float2(0.f, 0.f);
  }
  double dc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) dc[j] = 0.0;
  const int64_t kstride = (int64_t)nc * NY;
  for (int kd = kd_a; kd < kd_b; ++kd) {
    const double2 k = kc[kd];
    const bool near = ct_ok && (fabs(k.x - ctx) < o.r || (ct_m && fabs(k.x + ctx) < o.r));
    if (!__ballot(near)) {
      if (lane == 0) pdth[(int64_t)cs * n_k + kd] = 0.f;
      continue;
    }
    float2 v[16];
    const float2* xcol = X + kd * kstride + (int64_t)c0 * NY;
    if (g_stored) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, m;
        fft_out_index<NY>(lane, i, b, m);
        v[i] = (c0 + b < nc) ? xcol[(int64_t)b * NY + m] : make_float2(0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int b, n;
        fft_in_index<NY>(lane, i, b, n);
        v[i] = (c0 + b < nc) ? xcol[(int64_t)b * NY + n] : make_float2(0.f, 0.f);
      }
      wave_fft<NY>(v, buf, s_tw, lane);
    }
    const double kch = kchi[kd];
    const float kxf = (float)k.x, kyf = (float)k.y;
    double bk[8];
    chi_basis(k.x, k.y, o, bk);
    float wsum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int b, m;
      fft_out_index<NY>(lane, i, b, m);
      int c = c0 + b;
      asm volatile("" : "+v"(c), "+v"(m));  // see k_yreduce
      if (c >= nc) continue;
      for (int side = 0; side < 2; ++side) {
        int ix, iy;
        if (side == 0) {
          ix = signed_index(c, nx);
          iy = signed_index(m, NY);
        } else {
          if (!(c > 0 && 2 * c < nx)) break;
          ix = signed_index(nx - c, nx);
          iy = signed_index((NY - m) & (NY - 1), NY);
        }
        if (!overlap_screened(k.x, k.y, kxf, kyf, ix, iy, o)) continue;
        const double qx = (double)ix * o.sx, qy = (double)iy * o.sy;
        double bm[8];
        chi_basis(k.x - qx, k.y - qy, o, bm);
        double chim = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) chim += o.c[j] * bm[j];
        const float2 e = expi_reduced(chim - kch);
        const float2 gq = side ? cconj(v[i]) : v[i];
        const float2 z = make_float2(gq.x * e.x - gq.y * e.y, gq.x * e.y + gq.y * e.x);
        const float2 tb = side ? tbm[i] : tbd[i];
        const float w = tb.x * (-z.y) + tb.y * z.x;
        wsum += w;
#pragma unroll
        for (int j = 0; j < 8; ++j) dc[j] += (double)w * (bm[j] - bk[j]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
    if (lane == 0) pdth[(int64_t)cs * n_k + kd] = -wsum;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double v = dc[j];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) pdc[wid * 8 + j] = v;
  }
}

static int launch_yadjoint(int ny, const float2* X, const double2* kc, const double* kchi, int n_k, int nx,
                           int ngroups, const Optics& o, int g_stored, const float2* Tbt, double* pdc,
                           float* pdth, hipStream_t s) {
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  const dim3 grid((unsigned)(((ncs + 3) / 4) * ngroups)), blk(kYThreads);
  STEM_TRACE("ssb_yadjoint", s);
  switch (ny) {
    case 32: hipLaunchKernelGGL((k_yadjoint<32>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    case 64: hipLaunchKernelGGL((k_yadjoint<64>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    case 128: hipLaunchKernelGGL((k_yadjoint<128>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    case 256: hipLaunchKernelGGL((k_yadjoint<256>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    case 512: hipLaunchKernelGGL((k_yadjoint<512>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    case 1024: hipLaunchKernelGGL((k_yadjoint<1024>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, g_stored, Tbt, pdc, pdth); break;
    default: return STEM_EINVAL;
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

static int launch_yreduce(int ny, float2* X, const double2* kc, const double* kchi, int n_k, int nx,
                          int ngroups, const Optics& o, int store_g, float2* part,
                          unsigned long long* stats, hipStream_t s) {
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  const dim3 grid((unsigned)(((ncs + 3) / 4) * ngroups)), blk(kYThreads);
  STEM_TRACE("ssb_yreduce", s);
  switch (ny) {
    case 32: hipLaunchKernelGGL((k_yreduce<32>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    case 64: hipLaunchKernelGGL((k_yreduce<64>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    case 128: hipLaunchKernelGGL((k_yreduce<128>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    case 256: hipLaunchKernelGGL((k_yreduce<256>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    case 512: hipLaunchKernelGGL((k_yreduce<512>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    case 1024: hipLaunchKernelGGL((k_yreduce<1024>), grid, blk, 0, s, X, kc, kchi, n_k, nx, ngroups, o, store_g, part, stats); break;
    default: return STEM_EINVAL;
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// number of pixel groups of the fused sum: about 4096 waves, at most n_k, partial sums <= 64 MB
static int yreduce_groups(int ny, int nx, int n_k) {
  const int B = 1024 / ny;
  const int ncs = (nx / 2 + 1 + B - 1) / B;
  int g = (4096 + ncs - 1) / ncs;
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
// sums the adjoint partials in a fixed order: dL/dc over waves, dL/dtheta over column sets

__global__ void __launch_bounds__(256) k_adjoint_final(const double* __restrict__ pdc, int64_t npdc,
                                                       const float* __restrict__ pdth, int64_t npdth, int n_k,
                                                       double* __restrict__ dLdc, float* __restrict__ dLdth) {
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
  if (dLdth)
    for (int kd = threadIdx.x; kd < n_k; kd += blockDim.x) {
      double a = 0.0;
      for (int64_t b = 0; b < npdth; ++b) a += (double)pdth[b * n_k + kd];
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
  optics_poly(o);
  optics_screen(o, sc.ny, sc.nx);
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
  float2* part;
};

static Bufs carve(void* state, const SsbLayout& L) {
  char* p = (char*)state;
  return Bufs{(RowRun*)(p + L.rows), (double2*)(p + L.kc), (double*)(p + L.kchi),
              (unsigned long long*)(p + L.stats), (void*)(p + L.D),
              (float2*)(p + L.X),    (float2*)(p + L.T),  (float2*)(p + L.A),     (float2*)(p + L.Tb),
              (double*)(p + L.pdc),  (float*)(p + L.pdth), (float2*)(p + L.part)};
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
  if ((st = run_chi_table(b, d_theta, n_k, o, (mode == STEM_SSB_REFOCUS || ssb->normalize) ? 1 : L.groups, s)))
    return st;
  if (mode == STEM_SSB_REFOCUS) {
    // Eq. 3 again from the stored G
    if ((st = run_reduce_stored(L, b, ny, nx, o, ssb->normalize, s))) return st;
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
  if ((st = launch_yreduce(ny, b.X, b.kc, b.kchi, n_k, nx, L.groups, o, ssb->g_mode == STEM_G_STORE, b.part,
                           b.stats, s)))
    return st;
  return run_phase(L, b, *scan, b.part, L.groups, d_phase, d_T, s);
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
  if ((st = run_chi_table(b, d_theta, n_k, o, L.groups, s))) return st;
  if ((st = launch_yadjoint(ny, b.X, b.kc, b.kchi, n_k, nx, L.groups, o, ssb->g_mode == STEM_G_STORE, b.Tb, b.pdc,
                            b.pdth, s)))
    return st;
  {
    STEM_TRACE("ssb_adjoint_final", s);
    hipLaunchKernelGGL(k_adjoint_final, dim3(1), dim3(256), 0, s, b.pdc, L.nwy, b.pdth, (int64_t)L.ncs, n_k, d_dLdc,
                       d_dLdtheta);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
