// Event ingest and per-frame event reductions on linear-index EER (Sec. II, Table 1, Eq. 4).
//
//  k_validate       : range check of event indices and monotonicity of frame offsets.
//  k_com            : per-frame count and exact integer first moments -> centre of mass.
//  k_bin            : per-frame binned, cropped counts into the dense cube D[kd][f].
//
// Frame blocks: a workgroup owns a run of consecutive frames; their events are one
// contiguous CSR slice, streamed into LDS with coalesced loads in windows of kWin events.
#include "common.h"
#include "geom.h"
#include "kernels.h"
#include "trace.h"

namespace stem {

constexpr int kComThreads = 256;   // one frame per thread
constexpr int kWin = 4096;         // events per LDS window

// ---------------------------------------------------------------------------------------------
// validation

// Events are only read inside [lo_bound, hi_bound), the range the caller guarantees to be
// allocated; offsets outside it are reported, never followed.
__global__ void __launch_bounds__(256) k_validate(const int32_t* __restrict__ idx,
                                                  const int64_t* __restrict__ off, int64_t frame0,
                                                  int64_t n_frames, int64_t n_events, int exact_count,
                                                  int64_t lo_bound, int64_t hi_bound, int32_t npix,
                                                  int32_t* status) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = off[frame0];
  const int64_t e1 = off[frame0 + n_frames];
  int32_t bits = 0;
  const bool bounds_ok = e0 >= lo_bound && e0 <= e1 && e1 <= hi_bound;
  if (tid == 0 && (!bounds_ok || (exact_count && e1 - e0 != n_events))) bits |= STEM_EOFFSETS;
  for (int64_t f = tid; f < n_frames; f += nthr)
    if (off[frame0 + f + 1] < off[frame0 + f]) bits |= STEM_EOFFSETS;
  if (bounds_ok) {
    for (int64_t e = e0 + tid; e < e1; e += nthr) {
      const int32_t k = idx[e];
      if (k < 0 || k >= npix) bits |= STEM_ERANGE;
    }
  }
  int32_t wbits = bits;
  for (int o = 32; o > 0; o >>= 1) wbits |= __shfl_xor(wbits, o);
  if ((threadIdx.x & 63) == 0 && wbits) report(status, wbits);
}

// ---------------------------------------------------------------------------------------------
// centre of mass

__global__ void __launch_bounds__(kComThreads) k_com(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off,
                                                     int64_t frame0, int64_t n_frames, Magic divw,
                                                     int32_t cx, int32_t cy, int32_t npix,
                                                     int64_t nplane, double* __restrict__ com64,
                                                     float* __restrict__ com32,
                                                     int32_t* __restrict__ counts,
                                                     int32_t* status) {
  __shared__ int64_t s_off[kComThreads + 1];
  __shared__ int32_t s_ev[kWin];
  const int t = threadIdx.x;
  const int64_t fb = frame0 + (int64_t)blockIdx.x * kComThreads;  // first frame of the block
  const int64_t fend = frame0 + n_frames;
  const int nf = (int)((fend - fb) < kComThreads ? (fend - fb) : kComThreads);
  for (int i = t; i <= nf; i += kComThreads) s_off[i] = off[fb + i];
  __syncthreads();
  const int64_t ebeg = s_off[0], eend = s_off[nf];
  const int64_t my_lo = t < nf ? s_off[t] : 0, my_hi = t < nf ? s_off[t + 1] : 0;
  int64_t sx = 0, sy = 0;
  int32_t bad = 0;
  for (int64_t w0 = ebeg; w0 < eend; w0 += kWin) {
    const int wn = (int)((eend - w0) < kWin ? (eend - w0) : kWin);
    __syncthreads();
    for (int i = t; i < wn; i += kComThreads) s_ev[i] = idx[w0 + i];
    __syncthreads();
    const int64_t lo = my_lo > w0 ? my_lo : w0;
    const int64_t hi = my_hi < w0 + wn ? my_hi : w0 + wn;
    for (int64_t e = lo; e < hi; ++e) {
      const int32_t k = s_ev[e - w0];
      if (k < 0 || k >= npix) {
        bad = STEM_ERANGE;
        continue;
      }
      const uint32_t ky = magic_div((uint32_t)k, divw);
      const int32_t kx = k - (int32_t)(ky * divw.d);
      sx += kx - cx;
      sy += (int32_t)ky - cy;
    }
  }
  if (t < nf) {
    const int64_t f = fb + t;
    const int64_t n = my_hi - my_lo;
    const double x = n > 0 ? (double)sx / (double)n : 0.0;
    const double y = n > 0 ? (double)sy / (double)n : 0.0;
    if (com64) {
      com64[f] = x;
      com64[nplane + f] = y;
    }
    if (com32) {
      com32[f] = (float)x;
      com32[nplane + f] = (float)y;
    }
    if (counts) counts[f] = (int32_t)(n < 0x7fffffff ? n : 0x7fffffff);
  }
  if (bad) report(status, bad);
}

int launch_com(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, int64_t nplane, double* com64, float* com32, int32_t* counts,
               int32_t* status, hipStream_t stream) {
  if (n_frames == 0) return STEM_OK;
  const int64_t blocks = (n_frames + kComThreads - 1) / kComThreads;
  STEM_TRACE("com_moments", stream);
  hipLaunchKernelGGL(k_com, dim3((unsigned)blocks), dim3(kComThreads), 0, stream, idx, off, frame0,
                     n_frames, make_magic((uint32_t)det.W), det.cx, det.cy, det.W * det.H, nplane,
                     com64, com32, counts, status);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// geometry of the kept set (one workgroup)

__global__ void __launch_bounds__(256) k_geometry(int32_t b, int32_t nbx, int32_t nby, int32_t cx,
                                                  int32_t cy, double r2, RowRun* __restrict__ rows,
                                                  double2* __restrict__ kc) {
  __shared__ int32_t s_lo[1024];
  __shared__ int32_t s_hi[1024];
  __shared__ int32_t s_start[1024];
  __shared__ int32_t s_base;
  if (threadIdx.x == 0) s_base = 0;
  // nby <= 4096 is checked on the host; rows are handled in slices of 1024
  for (int r0 = 0; r0 < nby; r0 += 1024) {
    const int nr = nby - r0 < 1024 ? nby - r0 : 1024;
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      int lo, hi;
      kept_run(b, r0 + r, nbx, cx, cy, r2, lo, hi);
      s_lo[r] = lo;
      s_hi[r] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t base = s_base;
      for (int r = 0; r < nr; ++r) {
        s_start[r] = base;  // exclusive prefix of the run lengths
        base += s_hi[r] - s_lo[r];
      }
      s_base = base;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
      RowRun rr;
      rr.start = s_start[r];
      rr.lo = s_lo[r];
      rr.hi = s_hi[r];
      rr.pad = 0;
      rows[r0 + r] = rr;
      const double ky = bin_centre(b, r0 + r, cy);
      for (int bx = rr.lo; bx < rr.hi; ++bx)
        kc[rr.start + bx - rr.lo] = make_double2(bin_centre(b, bx, cx), ky);
    }
    __syncthreads();
  }
}

int launch_geometry(const stem_det& det, double r2, RowRun* rows, double2* kc, hipStream_t stream) {
  const int nbx = det.W / det.bin, nby = det.H / det.bin;
  STEM_TRACE("ssb_geometry", stream);
  hipLaunchKernelGGL(k_geometry, dim3(1), dim3(256), 0, stream, det.bin, nbx, nby, det.cx, det.cy, r2,
                     rows, kc);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// binning into D[kd][f] (frames of whole scan rows)
//
// Workgroup = (block of kBinFrames frames) x (run of kBinChunk kept pixels).  Counters are
// 16-bit, two per LDS word (frames fl and fl+1 of one pixel share a word).  A frame with
// more than 65535 events could carry into its neighbour and is rejected (STEM_EOVERFLOW).

constexpr int kBinFrames = 256;
constexpr int kBinChunk = 64;
constexpr int kBinThreads = 256;

template <typename DT>
__global__ void __launch_bounds__(kBinThreads) k_bin(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off, int64_t frame0,
                                                     int64_t n_frames, Magic divw, Magic divb,
                                                     int32_t npix, int32_t nby,
                                                     const RowRun* __restrict__ rows, int32_t n_k,
                                                     int64_t F, DT* __restrict__ D, int32_t* status) {
  __shared__ uint32_t s_hist[kBinChunk * kBinFrames / 2];
  __shared__ int64_t s_off[kBinFrames + 1];
  __shared__ int32_t s_ev[kWin];
  const int t = threadIdx.x;
  const int nchunks = (n_k + kBinChunk - 1) / kBinChunk;
  const int kd0 = (int)(blockIdx.x % nchunks) * kBinChunk;
  const int64_t fb = frame0 + (int64_t)(blockIdx.x / nchunks) * kBinFrames;
  const int64_t fend = frame0 + n_frames;
  const int nf = (int)((fend - fb) < kBinFrames ? (fend - fb) : kBinFrames);
  const int nkc = n_k - kd0 < kBinChunk ? n_k - kd0 : kBinChunk;
  for (int i = t; i < kBinChunk * kBinFrames / 2; i += kBinThreads) s_hist[i] = 0u;
  for (int i = t; i <= nf; i += kBinThreads) s_off[i] = off[fb + i];
  __syncthreads();
  int32_t bad = 0;
  if (t < nf && s_off[t + 1] - s_off[t] > 65535) bad |= STEM_EOVERFLOW;
  const int64_t ebeg = s_off[0], eend = s_off[nf];
  const int64_t my_lo = t < nf ? s_off[t] : 0, my_hi = t < nf ? s_off[t + 1] : 0;
  for (int64_t w0 = ebeg; w0 < eend; w0 += kWin) {
    const int wn = (int)((eend - w0) < kWin ? (eend - w0) : kWin);
    __syncthreads();
    for (int i = t; i < wn; i += kBinThreads) s_ev[i] = idx[w0 + i];
    __syncthreads();
    // thread t bins the events of frame t that fall in this window
    const int64_t lo = my_lo > w0 ? my_lo : w0;
    const int64_t hi = my_hi < w0 + wn ? my_hi : w0 + wn;
    for (int64_t e = lo; e < hi; ++e) {
      const int32_t k = s_ev[e - w0];
      if (k < 0 || k >= npix) {
        bad |= STEM_ERANGE;
        continue;
      }
      const uint32_t ky = magic_div((uint32_t)k, divw);
      const uint32_t kx = (uint32_t)k - ky * divw.d;
      const int by = (int)magic_div(ky, divb);
      const int bx = (int)magic_div(kx, divb);
      if (by >= nby) continue;
      const RowRun rr = rows[by];
      if (bx < rr.lo || bx >= rr.hi) continue;
      const int kd = rr.start + bx - rr.lo - kd0;
      if (kd < 0 || kd >= nkc) continue;
      atomicAdd(&s_hist[(kd * kBinFrames + t) >> 1], (t & 1) ? 0x10000u : 1u);
    }
  }
  __syncthreads();
  // write out: each thread writes 2 consecutive frames of one pixel row per step
  const uint32_t cap = sizeof(DT) == 1 ? 255u : 65535u;
  for (int i = t; i < nkc * (kBinFrames / 2); i += kBinThreads) {
    const int kd = i / (kBinFrames / 2);
    const int fp = (i % (kBinFrames / 2)) * 2;
    if (fp >= nf) continue;
    const uint32_t w = s_hist[(kd * kBinFrames + fp) >> 1];
    const uint32_t c0 = w & 0xffffu, c1 = w >> 16;
    if (c0 > cap || c1 > cap) bad |= STEM_EOVERFLOW;
    DT* dst = D + (int64_t)(kd0 + kd) * F + (fb + fp);
    dst[0] = (DT)(c0 > cap ? cap : c0);
    if (fp + 1 < nf) dst[1] = (DT)(c1 > cap ? cap : c1);
  }
  if (bad) report(status, bad);
}

int launch_bin(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, const RowRun* rows, int n_k, int64_t F, void* D, int d_bits,
               int32_t* status, hipStream_t stream) {
  if (n_frames == 0) return STEM_OK;
  const int nchunks = (n_k + kBinChunk - 1) / kBinChunk;
  const int64_t fblocks = (n_frames + kBinFrames - 1) / kBinFrames;
  const dim3 grid((unsigned)(fblocks * nchunks));
  const Magic mw = make_magic((uint32_t)det.W), mb = make_magic((uint32_t)det.bin);
  const int nby = det.H / det.bin;
  STEM_TRACE("bin_densify", stream);
  if (d_bits == 8)
    hipLaunchKernelGGL(k_bin<uint8_t>, grid, dim3(kBinThreads), 0, stream, idx, off, frame0, n_frames, mw,
                       mb, det.W * det.H, nby, rows, n_k, F, (uint8_t*)D, status);
  else
    hipLaunchKernelGGL(k_bin<uint16_t>, grid, dim3(kBinThreads), 0, stream, idx, off, frame0, n_frames,
                       mw, mb, det.W * det.H, nby, rows, n_k, F, (uint16_t*)D, status);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

}  // namespace stem

// ---------------------------------------------------------------------------------------------
// C ABI

using namespace stem;

extern "C" const char* stem_strerror(int status) {
  switch (status) {
    case STEM_OK: return "ok";
    case STEM_EINVAL: return "invalid argument";
    case STEM_ERANGE: return "event index outside the detector";
    case STEM_EOFFSETS: return "frame offsets not monotone or inconsistent with the event count";
    case STEM_EOVERFLOW: return "binned count does not fit the element type";
    case STEM_EWORKSPACE: return "workspace or state buffer too small or misaligned";
    case STEM_EHIP: return "HIP runtime error";
    case STEM_ESTATE: return "state buffer not prepared for this mode";
    default: return "several errors (status bits)";
  }
}

extern "C" int stem_version(void) { return 100; }

extern "C" int eer_load_csr(const int32_t* h_idx, const int64_t* h_off, int64_t frame0,
                            int64_t n_frames, int64_t n_events, const stem_det* det, int32_t* d_idx,
                            int64_t* d_off, int32_t* d_status, void* stream_) {
  if (!det || !d_idx || !d_off || frame0 < 0 || n_frames < 0 || n_events < 0) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  if ((h_idx == nullptr) != (h_off == nullptr)) return STEM_EINVAL;
  hipStream_t stream = (hipStream_t)stream_;
  if (h_off) {
    if (h_off[0] < 0 || h_off[n_frames] - h_off[0] != n_events) return STEM_EINVAL;
    STEM_HIP_CHECK(hipMemcpyAsync(d_off + frame0, h_off, sizeof(int64_t) * (n_frames + 1),
                                  hipMemcpyHostToDevice, stream));
    if (n_events > 0)
      STEM_HIP_CHECK(hipMemcpyAsync(d_idx + h_off[0], h_idx, sizeof(int32_t) * n_events,
                                    hipMemcpyHostToDevice, stream));
  }
  // copy mode: the chunk's events occupy exactly [h_off[0], h_off[0] + n_events);
  // validate-only mode: d_idx holds n_events entries and the chunk must lie inside them
  const int64_t lo = h_off ? h_off[0] : 0;
  const int64_t hi = h_off ? h_off[0] + n_events : n_events;
  int64_t work = n_frames > n_events ? n_frames : n_events;
  int64_t blocks = (work + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  {
    STEM_TRACE("csr_validate", stream);
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, stream, d_idx, d_off, frame0,
                       n_frames, n_events, h_off ? 1 : 0, lo, hi, det->W * det->H, d_status);
  }
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
