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
// block-local frame lookup shared by the event-parallel kernels

// Loads the block's offsets relative to its first event.  Returns false (and reports) when
// the block holds 2^30 events or more, which the 32-bit relative offsets cannot address.
__device__ __forceinline__ bool load_rel_offsets(const int64_t* __restrict__ off, int64_t fb, int nf,
                                                 int32_t* s_rel, int64_t* s_base, int32_t* status) {
  const int64_t base = off[fb];
  const int64_t span = off[fb + nf] - base;
  if (span >= (1ll << 30)) {
    if (threadIdx.x == 0) report(status, STEM_EOVERFLOW);
    return false;
  }
  for (int i = threadIdx.x; i <= nf; i += blockDim.x) s_rel[i] = (int32_t)(off[fb + i] - base);
  if (threadIdx.x == 0) *s_base = base;
  return true;
}

// ---------------------------------------------------------------------------------------------
// Thread-per-frame walk over a frame's events: a scalar head up to 16-byte alignment, then
// 16-byte vector loads (four events each, four loads issued together), then a scalar tail.
// f(k) is applied to every event index in order.

template <typename Fn>
__device__ __forceinline__ void for_each_event(const int32_t* __restrict__ ev, int64_t lo, int64_t hi, Fn f) {
  int64_t e = lo;
  for (; e < hi && (((uintptr_t)(ev + e)) & 15); ++e) f(ev[e]);
  for (; e + 16 <= hi; e += 16) {
    const int4 q0 = *(const int4*)(ev + e);
    const int4 q1 = *(const int4*)(ev + e + 4);
    const int4 q2 = *(const int4*)(ev + e + 8);
    const int4 q3 = *(const int4*)(ev + e + 12);
    f(q0.x); f(q0.y); f(q0.z); f(q0.w);
    f(q1.x); f(q1.y); f(q1.z); f(q1.w);
    f(q2.x); f(q2.y); f(q2.z); f(q2.w);
    f(q3.x); f(q3.y); f(q3.z); f(q3.w);
  }
  for (; e + 4 <= hi; e += 4) {
    const int4 q = *(const int4*)(ev + e);
    f(q.x); f(q.y); f(q.z); f(q.w);
  }
  for (; e < hi; ++e) f(ev[e]);
}

// ---------------------------------------------------------------------------------------------
// centre of mass: one thread per frame

__global__ void __launch_bounds__(kComThreads) k_com(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off,
                                                     int64_t frame0, int64_t n_frames, Magic divw,
                                                     int32_t cx, int32_t cy, int32_t npix,
                                                     int64_t nplane, double* __restrict__ com64,
                                                     float* __restrict__ com32,
                                                     int32_t* __restrict__ counts,
                                                     int32_t* status) {
  const int64_t fr = frame0 + (int64_t)blockIdx.x * kComThreads + threadIdx.x;
  if (fr >= frame0 + n_frames) return;
  const int64_t lo = off[fr], hi = off[fr + 1];
  int64_t sx = 0, sy = 0;
  int32_t bad = 0;
  for_each_event(idx, lo, hi, [&](int32_t k) {
    if (k < 0 || k >= npix) {
      bad = STEM_ERANGE;
      return;
    }
    const uint32_t ky = magic_div((uint32_t)k, divw);
    sx += k - (int32_t)(ky * divw.d) - cx;
    sy += (int32_t)ky - cy;
  });
  const int64_t n = hi - lo;
  const double x = n > 0 ? (double)sx / (double)n : 0.0;
  const double y = n > 0 ? (double)sy / (double)n : 0.0;
  if (com64) {
    com64[fr] = x;
    com64[nplane + fr] = y;
  }
  if (com32) {
    com32[fr] = (float)x;
    com32[nplane + fr] = (float)y;
  }
  if (counts) counts[fr] = (int32_t)(n < 0x7fffffff ? n : 0x7fffffff);
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
// Workgroup = kBinFrames consecutive frames x a run of up to kBinKd kept pixels.  Events are
// processed in parallel (coalesced loads, frame by binary search in the block's offsets) and
// counted in LDS: 8-bit counters, four frames per word, when every frame of the block has at
// most 255 events (no count can then carry into its neighbour); otherwise 16-bit counters, two
// frames per word, over two passes of half the pixels.  A count above the element type of D
// sets STEM_EOVERFLOW (the stored value is then not meaningful).

constexpr int kBinFrames = 256;
constexpr int kBinThreads = 256;
constexpr int kBinWords = 11776;                      // 46 KB of counters
// pixel rows of counters are kBinFrames/4 (+1 padding) words apart, so that the events of one
// frame (same column, different pixels) fall into different LDS banks
constexpr int kBinKd = kBinWords / (kBinFrames / 4 + 1);  // 181 pixels per workgroup
constexpr int kBinLdsRows = 256;                      // bin rows cached in LDS

template <typename DT>
__global__ void __launch_bounds__(kBinThreads) k_bin(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off, int64_t frame0,
                                                     int64_t n_frames, Magic divw, Magic divb,
                                                     int32_t npix, int32_t nby,
                                                     const RowRun* __restrict__ rows, int32_t n_k,
                                                     int64_t F, DT* __restrict__ D, int32_t* status) {
  __shared__ uint32_t s_hist[kBinWords];
  __shared__ int32_t s_rel[kBinFrames + 1];
  __shared__ RowRun s_rows[kBinLdsRows];
  __shared__ int64_t s_base;
  const int t = threadIdx.x;
  const int nchunks = (n_k + kBinKd - 1) / kBinKd;
  const int kd0 = (int)(blockIdx.x % nchunks) * kBinKd;
  const int kc = n_k - kd0 < kBinKd ? n_k - kd0 : kBinKd;
  const int64_t fb = frame0 + (int64_t)(blockIdx.x / nchunks) * kBinFrames;
  const int64_t fend = frame0 + n_frames;
  const int nf = (int)((fend - fb) < kBinFrames ? (fend - fb) : kBinFrames);
  if (!load_rel_offsets(off, fb, nf, s_rel, &s_base, status)) return;
  const bool rows_lds = nby <= kBinLdsRows;
  if (rows_lds)
    for (int i = t; i < nby; i += kBinThreads) s_rows[i] = rows[i];
  __syncthreads();
  const int wide = __syncthreads_or(t < nf && s_rel[t + 1] - s_rel[t] > 255);
  const int32_t* ev = idx + s_base;
  const RowRun* rtab = rows_lds ? s_rows : rows;
  int32_t bad = 0;
  const int npass = wide ? 2 : 1;
  const int kpp = (kc + npass - 1) / npass;       // pixels per pass
  const int fpw = wide ? 2 : 4;                   // frames per counter word
  const int wpr = kBinFrames / fpw;               // words per pixel row
  const int wps = wpr + 1;                        // row stride in words (padded)
  const uint32_t cap = sizeof(DT) == 1 ? 255u : 65535u;
  for (int pass = 0; pass < npass; ++pass) {
    const int ka = kd0 + pass * kpp;
    const int kn = (kd0 + kc) - ka < kpp ? (kd0 + kc) - ka : kpp;
    for (int i = t; i < kn * wps; i += kBinThreads) s_hist[i] = 0u;
    __syncthreads();
    // thread t walks the events of frame t
    if (t < nf) {
      const int shift = wide ? 16 * (t & 1) : 8 * (t & 3);
      const int col = wide ? (t >> 1) : (t >> 2);
      for_each_event(ev, s_rel[t], s_rel[t + 1], [&](int32_t k) {
        if (k < 0 || k >= npix) {
          bad |= STEM_ERANGE;
          return;
        }
        const uint32_t ky = magic_div((uint32_t)k, divw);
        const uint32_t kx = (uint32_t)k - ky * divw.d;
        const int by = (int)magic_div(ky, divb);
        const int bx = (int)magic_div(kx, divb);
        if (by >= nby) return;
        const RowRun rr = rtab[by];
        if (bx < rr.lo || bx >= rr.hi) return;
        const int kd = rr.start + bx - rr.lo - ka;
        if (kd < 0 || kd >= kn) return;
        atomicAdd(&s_hist[kd * wps + col], 1u << shift);
      });
    }
    __syncthreads();
    // one counter word per thread and step: fpw consecutive frames of one pixel row
    for (int i = t; i < kn * wpr; i += kBinThreads) {
      const int kd = i / wpr, q = i % wpr;
      const int f0 = q * fpw;
      if (f0 >= nf) continue;
      const uint32_t w = s_hist[kd * wps + q];
      uint32_t c[4];
      if (wide) {
        c[0] = w & 0xffffu;
        c[1] = w >> 16;
        c[2] = c[3] = 0u;
      } else {
        c[0] = w & 0xffu;
        c[1] = (w >> 8) & 0xffu;
        c[2] = (w >> 16) & 0xffu;
        c[3] = w >> 24;
      }
      DT* dst = D + (int64_t)(ka + kd) * F + (fb + f0);
      if (f0 + fpw <= nf) {
        if (sizeof(DT) == 1 && !wide) {
          *(uint32_t*)dst = w;  // four 8-bit counts are the four bytes
        } else {
          for (int j = 0; j < fpw; ++j) {
            if (c[j] > cap) bad |= STEM_EOVERFLOW;
            dst[j] = (DT)c[j];
          }
        }
      } else {
        for (int j = 0; j < fpw && f0 + j < nf; ++j) {
          if (c[j] > cap) bad |= STEM_EOVERFLOW;
          dst[j] = (DT)c[j];
        }
      }
    }
    __syncthreads();
  }
  if (bad) report(status, bad);
}

int launch_bin(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, const RowRun* rows, int n_k, int64_t F, void* D, int d_bits,
               int32_t* status, hipStream_t stream) {
  if (n_frames == 0) return STEM_OK;
  const int nchunks = (n_k + kBinKd - 1) / kBinKd;
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
