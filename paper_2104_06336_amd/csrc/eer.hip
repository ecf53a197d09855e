// Event ingest and per-frame event reductions on linear-index EER (Sec. II, Table 1, Eq. 4).
//
//  k_validate       : range check of event indices and monotonicity of frame offsets.
//  k_com            : per-frame count and exact integer first moments -> centre of mass.
//  k_bin            : per-frame binned, cropped counts into the dense cube D[kd][f].
//
// Frame blocks: a workgroup owns a run of consecutive frames; their events are one contiguous
// CSR slice, read with coalesced 16-byte loads: staged in LDS for the per-frame sums of k_com,
// streamed with an LDS map event -> frame for the counts of k_bin.
#include <cmath>
#include <type_traits>

#include "common.h"
#include "geom.h"
#include "kernels.h"
#include "optics.h"
#include "trace.h"

namespace stem {

constexpr int kComThreads = 256;   // = kComFrames: thread t finishes frame t

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
// Group c of four events starting at the absolute index e (16-byte aligned): k[j] = idx[e + j],
// ok[j] = e + j in [a0, aend); the whole group is one 16-byte load when it lies inside.
__device__ __forceinline__ void load_group(const int32_t* __restrict__ idx, int64_t e, int64_t a0, int64_t aend,
                                           int32_t* k, bool* ok) {
  if (e >= a0 && e + 4 <= aend) {
    const int4 v = *(const int4*)(idx + e);
    k[0] = v.x;
    k[1] = v.y;
    k[2] = v.z;
    k[3] = v.w;
#pragma unroll
    for (int j = 0; j < 4; ++j) ok[j] = true;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ok[j] = e + j >= a0 && e + j < aend;
      k[j] = ok[j] ? idx[e + j] : 0;
    }
  }
}

// Staging of a workgroup's events in LDS: the events [a0, a0 + n) (absolute indices, n <= kComWin)
// are copied as whole 16-byte lines from the aligned position at or below a0; s[sh + j] then holds
// event a0 + j (sh < 4 is returned).  Every line holds at least one of the events, so it lies in
// the event array's pages; its other entries land outside [sh, sh + n) and are never read.  Each
// thread issues kStageGroups loads before its LDS stores: a window takes one round.
constexpr int kComWin = 12288;
constexpr int kStageGroups = kComWin / (4 * kComThreads);

__device__ __forceinline__ int stage_events(const int32_t* __restrict__ idx, int64_t a0, int n, int32_t* s) {
  const int sh = (int)((((uintptr_t)(idx + a0)) & 15) >> 2);
  const int32_t* ib = idx + (a0 - sh);
  const int ng = (n + sh + 3) >> 2;
  for (int c0 = threadIdx.x; c0 < ng; c0 += kComThreads * kStageGroups) {
    int4 v[kStageGroups];
#pragma unroll
    for (int u = 0; u < kStageGroups; ++u) {
      const int c = c0 + u * kComThreads;
      v[u] = c < ng ? *(const int4*)(ib + 4 * c) : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < kStageGroups; ++u) {
      const int c = c0 + u * kComThreads;
      if (c < ng) *(int4*)&s[4 * c] = v[u];
    }
  }
  return sh;
}

// ---------------------------------------------------------------------------------------------
// centre of mass: a workgroup owns kComFrames consecutive frames.  Their events are staged in
// LDS in windows of kComWin (coalesced 16-byte loads); thread t then sums the events of frame t
// from LDS with four independent accumulators (int32 within a window, int64 across windows).

constexpr int kComFrames = 256;

__global__ void __launch_bounds__(kComThreads) k_com(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off,
                                                     int64_t frame0, int64_t n_frames, Magic divw,
                                                     int32_t cx, int32_t cy, int32_t npix,
                                                     int64_t nplane, double* __restrict__ com64,
                                                     float* __restrict__ com32,
                                                     int32_t* __restrict__ counts,
                                                     int32_t* status) {
  __shared__ __align__(16) int32_t s_ev[kComWin + 8];
  __shared__ int32_t s_rel[kComFrames + 1];
  __shared__ int64_t s_base;
  const int t = threadIdx.x;
  const int64_t fb = frame0 + (int64_t)blockIdx.x * kComFrames;
  const int64_t left = frame0 + n_frames - fb;
  const int nf = (int)(left < kComFrames ? left : kComFrames);
  if (!load_rel_offsets(off, fb, nf, s_rel, &s_base, status)) return;
  __syncthreads();
  const int span = s_rel[nf];
  const int lo_t = t < nf ? s_rel[t] : 0, hi_t = t < nf ? s_rel[t + 1] : 0;
  int64_t sx = 0, sy = 0;
  int32_t bad = 0;
  for (int w0 = 0; w0 < span; w0 += kComWin) {
    const int wn = span - w0 < kComWin ? span - w0 : kComWin;
    __syncthreads();
    const int sh = stage_events(idx, s_base + w0, wn, s_ev);
    __syncthreads();
    const int lo = (lo_t > w0 ? lo_t : w0) - w0 + sh;
    const int hi = (hi_t < w0 + wn ? hi_t : w0 + wn) - w0 + sh;
    int32_t ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
    uint32_t nbad = 0;
    // out-of-range indices are counted (and reported) and contribute nothing; no branches
    auto add = [&](int j, int32_t k) {
      const bool in = (uint32_t)k < (uint32_t)npix;
      nbad += in ? 0u : 1u;
      const uint32_t kk = in ? (uint32_t)k : 0u;
      const uint32_t ky = magic_div(kk, divw);
      ax[j] += in ? (int32_t)(kk - ky * divw.d) - cx : 0;
      ay[j] += in ? (int32_t)ky - cy : 0;
    };
    int e = lo;
    for (; e + 4 <= hi; e += 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j) add(j, s_ev[e + j]);
    }
    for (; e < hi; ++e) add(0, s_ev[e]);
    if (nbad) bad = STEM_ERANGE;
    sx += (int64_t)ax[0] + ax[1] + ax[2] + ax[3];
    sy += (int64_t)ay[0] + ay[1] + ay[2] + ay[3];
  }
  if (t < nf) {
    const int64_t fr = fb + t;
    const int64_t n = hi_t - lo_t;
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
    if (counts) counts[fr] = (int32_t)n;
  }
  if (bad) report(status, bad);
}

int launch_com(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, int64_t nplane, double* com64, float* com32, int32_t* counts,
               int32_t* status, hipStream_t stream) {
  if (n_frames == 0) return STEM_OK;
  const int64_t blocks = (n_frames + kComFrames - 1) / kComFrames;
  STEM_TRACE("com_moments", stream);
  hipLaunchKernelGGL(k_com, dim3((unsigned)blocks), dim3(kComThreads), 0, stream, idx, off, frame0,
                     n_frames, make_magic((uint32_t)det.W), det.cx, det.cy, det.W * det.H, nplane,
                     com64, com32, counts, status);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

// ---------------------------------------------------------------------------------------------
// virtual annular detectors: the same staging as k_com; thread t counts the events of frame t in
// each annulus [lo_j, hi_j) of squared pixel distance (exact int64 thresholds)

struct Annuli {
  int64_t lo[STEM_MAX_ANNULI], hi[STEM_MAX_ANNULI];
};

template <int NA>
__global__ void __launch_bounds__(kComThreads) k_annular(const int32_t* __restrict__ idx,
                                                         const int64_t* __restrict__ off, int64_t frame0,
                                                         int64_t n_frames, Magic divw, int32_t cx, int32_t cy,
                                                         int32_t npix, Annuli an, int64_t F,
                                                         int32_t* __restrict__ out, int32_t* status) {
  __shared__ __align__(16) int32_t s_ev[kComWin + 8];
  __shared__ int32_t s_rel[kComFrames + 1];
  __shared__ int64_t s_base;
  const int t = threadIdx.x;
  const int64_t fb = frame0 + (int64_t)blockIdx.x * kComFrames;
  const int64_t left = frame0 + n_frames - fb;
  const int nf = (int)(left < kComFrames ? left : kComFrames);
  if (!load_rel_offsets(off, fb, nf, s_rel, &s_base, status)) return;
  __syncthreads();
  const int span = s_rel[nf];
  const int lo_t = t < nf ? s_rel[t] : 0, hi_t = t < nf ? s_rel[t + 1] : 0;
  int32_t cnt[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) cnt[j] = 0;
  uint32_t nbad = 0;
  for (int w0 = 0; w0 < span; w0 += kComWin) {
    const int wn = span - w0 < kComWin ? span - w0 : kComWin;
    __syncthreads();
    const int sh = stage_events(idx, s_base + w0, wn, s_ev);
    __syncthreads();
    const int lo = (lo_t > w0 ? lo_t : w0) - w0 + sh;
    const int hi = (hi_t < w0 + wn ? hi_t : w0 + wn) - w0 + sh;
    for (int e = lo; e < hi; ++e) {
      const int32_t k = s_ev[e];
      const bool in = (uint32_t)k < (uint32_t)npix;
      nbad += in ? 0u : 1u;
      const uint32_t kk = in ? (uint32_t)k : 0u;
      const uint32_t ky = magic_div(kk, divw);
      const int64_t dx = (int64_t)(kk - ky * divw.d) - cx, dy = (int64_t)ky - cy;
      const int64_t d2 = dx * dx + dy * dy;
#pragma unroll
      for (int j = 0; j < NA; ++j) cnt[j] += (in && d2 >= an.lo[j] && d2 < an.hi[j]) ? 1 : 0;
    }
  }
  if (t < nf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) out[(int64_t)j * F + fb + t] = cnt[j];
  }
  if (nbad) report(status, STEM_ERANGE);
}

// ---------------------------------------------------------------------------------------------
// sum of frames: the event range is split evenly over the workgroups; each counts its events into
// 32-bit LDS counters over a box of up to 128 x 128 pixels around the zero-frequency pixel, where
// the bright-field disk and nearly all events fall (events outside the box go straight to global
// atomics), then adds the box to the global sum once.

constexpr int kSumBox = 128;
constexpr int kSumBlocks = 512;

__global__ void __launch_bounds__(256) k_sum_events(const int32_t* __restrict__ idx, const int64_t* __restrict__ off,
                                                    int64_t frame0, int64_t n_frames, Magic divw, int32_t npix,
                                                    int32_t bx0, int32_t by0, int32_t bw, int32_t bh,
                                                    uint32_t* __restrict__ sum, int32_t* status) {
  __shared__ uint32_t s_box[kSumBox * kSumBox];
  const int64_t e0 = off[frame0], e1 = off[frame0 + n_frames];
  if (e1 < e0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) report(status, STEM_EOFFSETS);
    return;
  }
  const int nbox = bw * bh;
  for (int i = threadIdx.x; i < nbox; i += blockDim.x) s_box[i] = 0u;
  __syncthreads();
  // this workgroup's share of the events, in whole 16-byte groups where possible
  const int64_t per = ((e1 - e0 + gridDim.x - 1) / gridDim.x + 3) & ~3ll;
  const int64_t a0 = e0 + (int64_t)blockIdx.x * per;
  const int64_t aend = a0 + per < e1 ? a0 + per : e1;
  uint32_t nbad = 0;
  if (a0 < aend) {
    const int sh = (int)((((uintptr_t)(idx + a0)) & 15) >> 2);
    const int64_t al = a0 - sh;
    const int64_t ng = (aend - al + 3) >> 2;
    constexpr int U = 4;  // groups per thread in flight
    for (int64_t g0 = threadIdx.x; g0 < ng; g0 += (int64_t)U * blockDim.x) {
      int32_t k[U][4];
      bool ok[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = g0 + (int64_t)u * blockDim.x;
        if (g < ng) {
          load_group(idx, al + 4 * g, a0, aend, k[u], ok[u]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            ok[u][q] = false;
            k[u][q] = 0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!ok[u][q]) continue;
          if ((uint32_t)k[u][q] >= (uint32_t)npix) {
            ++nbad;
            continue;
          }
          const uint32_t ky = magic_div((uint32_t)k[u][q], divw);
          const int x = (int)((uint32_t)k[u][q] - ky * divw.d) - bx0, y = (int)ky - by0;
          if ((uint32_t)x < (uint32_t)bw && (uint32_t)y < (uint32_t)bh)
            atomicAdd(&s_box[y * bw + x], 1u);
          else
            atomicAdd(&sum[k[u][q]], 1u);
        }
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < nbox; p += blockDim.x) {
    const uint32_t c = s_box[p];
    if (c) atomicAdd(&sum[(int64_t)(by0 + p / bw) * divw.d + bx0 + p % bw], c);
  }
  if (nbad) report(status, STEM_ERANGE);
}

__global__ void __launch_bounds__(256) k_frame_mean(const uint32_t* __restrict__ sum, int64_t npix, double n,
                                                    float* __restrict__ mean) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < npix) mean[p] = (float)((double)sum[p] / n);
}

// ---------------------------------------------------------------------------------------------
// run-length form -> linear indices: the block's distances are staged in LDS like k_com's
// events, thread t replaces its frame's distances by their running sum in place, and the
// workgroup writes the window back with 16-byte stores (the store groups that are not wholly
// inside the window are written element by element).

__global__ void __launch_bounds__(kComThreads) k_decode_rle(const int32_t* __restrict__ dist,
                                                            const int64_t* __restrict__ off, int64_t frame0,
                                                            int64_t n_frames, int32_t npix,
                                                            int32_t* __restrict__ idx, int32_t* status) {
  __shared__ __align__(16) int32_t s_ev[kComWin + 8];
  __shared__ int32_t s_rel[kComFrames + 1];
  __shared__ int64_t s_base;
  const int t = threadIdx.x;
  const int64_t fb = frame0 + (int64_t)blockIdx.x * kComFrames;
  const int64_t left = frame0 + n_frames - fb;
  const int nf = (int)(left < kComFrames ? left : kComFrames);
  if (!load_rel_offsets(off, fb, nf, s_rel, &s_base, status)) return;
  __syncthreads();
  const int span = s_rel[nf];
  const int lo_t = t < nf ? s_rel[t] : 0, hi_t = t < nf ? s_rel[t + 1] : 0;
  int64_t run = 0;  // running sum of frame t, carried across windows
  uint32_t nbad = 0;
  for (int w0 = 0; w0 < span; w0 += kComWin) {
    const int wn = span - w0 < kComWin ? span - w0 : kComWin;
    __syncthreads();
    const int sh = stage_events(dist, s_base + w0, wn, s_ev);
    __syncthreads();
    const int lo = (lo_t > w0 ? lo_t : w0) - w0 + sh;
    const int hi = (hi_t < w0 + wn ? hi_t : w0 + wn) - w0 + sh;
    for (int e = lo; e < hi; ++e) {
      run += s_ev[e];
      const bool in = run >= 0 && run < npix;
      nbad += in ? 0u : 1u;
      s_ev[e] = in ? (int32_t)run : -1;
    }
    __syncthreads();
    // write back [sh, sh + wn) of the staging buffer to idx[s_base + w0 ...]
    const int64_t a0 = s_base + w0, aend = a0 + wn, al = a0 - sh;
    const int nchunk = (wn + sh + 3) >> 2;
    for (int c = t; c < nchunk; c += blockDim.x) {
      const int64_t e = al + 4 * (int64_t)c;
      if (e >= a0 && e + 4 <= aend && ((((uintptr_t)(idx + e)) & 15) == 0)) {
        *(int4*)(idx + e) = *(const int4*)&s_ev[4 * c];
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (e + j >= a0 && e + j < aend) idx[e + j] = s_ev[4 * c + j];
      }
    }
  }
  if (nbad) report(status, STEM_ERANGE);
}

// ---------------------------------------------------------------------------------------------
// geometry of the kept set (one workgroup)

// The kept set's row runs and bin centres, by one workgroup of blockDim.x threads; s holds
// 3 * 1024 + 1 ints of LDS scratch.
__device__ void build_geometry(int32_t b, int32_t nbx, int32_t nby, int32_t cx, int32_t cy, double r2,
                               RowRun* __restrict__ rows, double2* __restrict__ kc, int32_t* s) {
  int32_t* s_lo = s;
  int32_t* s_hi = s + 1024;
  int32_t* s_start = s + 2048;
  int32_t& s_base = s[3072];
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

__global__ void __launch_bounds__(256) k_geometry(int32_t b, int32_t nbx, int32_t nby, int32_t cx,
                                                  int32_t cy, double r2, RowRun* __restrict__ rows,
                                                  double2* __restrict__ kc) {
  __shared__ int32_t s[3 * 1024 + 1];
  build_geometry(b, nbx, nby, cx, cy, r2, rows, kc, s);
}

// ---------------------------------------------------------------------------------------------
// pixel -> kept bin lookup: lut[ky*W + kx] = kd of the bin holding the pixel, -1 if that bin is
// dropped (its centre outside the disk)

__global__ void __launch_bounds__(256) k_pixel_lut(const RowRun* __restrict__ rows, int32_t W, int32_t H, int32_t b,
                                                   int16_t* __restrict__ lut) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)W * H) return;
  const int ky = (int)(p / W), kx = (int)(p % W);
  const RowRun rr = rows[ky / b];
  const int bx = kx / b;
  lut[p] = (int16_t)(bx >= rr.lo && bx < rr.hi ? rr.start + bx - rr.lo : -1);
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
// Workgroup = kBinFrames consecutive frames x a run of up to kBinKd kept pixels (small
// workgroups: several per CU hide the latency of their load, count and write-out phases).  The block's
// events are streamed in windows of kBinWin: first each thread writes its frame number into an
// LDS byte map over the window's events, then the events are read with coalesced 16-byte loads
// (four per lane), their frames read from the map as one word and their pixels mapped by the
// lookup table.  Counts live in LDS: 8-bit counters, four frames per word, when every frame of
// the block has at most 255 events (no count can then carry into its neighbour); otherwise
// 16-bit counters, two frames per word, over two passes of half the pixels.  A count above the
// element type of D sets STEM_EOVERFLOW (the stored value is then not meaningful).

constexpr int kBinFrames = 128;
constexpr int kBinThreads = 256;
constexpr int kBinWords = 5976;                       // 23 KB of counters
// pixel rows of counters are kBinFrames/4 (+1 padding) words apart, so that the events of one
// frame (same column, different pixels) fall into different LDS banks
constexpr int kBinKd = kBinWords / (kBinFrames / 4 + 1);  // 181 pixels per workgroup
constexpr int kBinWin = 6144;                         // events per window of the frame map (a block of
                                                      // 128 frames at 40 events per frame fits one)
constexpr int kBinBoxMax = 4096;                      // bins of the largest LDS bin table (8 KB)

// The kept bins' bounding box (in bins) and the divisions that take a pixel to its bin: with it
// (BOX) the pixel -> bin table is a small per-workgroup LDS copy over the box, looked up with a
// division by W (magic number) and by the binning (multiply-high), instead of a gather from the
// global per-pixel table.
constexpr int kBoxRows = 64;  // bin rows of the largest box whose row runs travel as arguments
struct BinBox {
  Magic mw;           // division by the detector width W
  uint32_t mbin;      // ceil(2^32 / bin); 0 for bin = 1
  int32_t W, bin;
  int32_t bx0, by0, bw, bh;
  int32_t start[kBoxRows], lo[kBoxRows], hi[kBoxRows];  // row runs of the box's rows (BOX)
};

// The kept set's geometry, written by the first workgroup of the binning kernel (BOX: the
// binning itself takes the box's row runs from its arguments)
struct GeomOut {
  RowRun* rows;       // nullptr: nothing to write
  double2* kc;
  int32_t nbx, nby, cx, cy;
  double r2;
  unsigned long long* mark;  // if set, cleared by the first thread (an accumulation from frame 0
                             // voids the state's FINALIZE)
};

// One step of a segmented inclusive scan within rows of 16 lanes: lane i adds the sums of lane
// i - d of its row when both hold the same key (sorted keys: equal keys are contiguous).  Lanes
// whose source lies before the row start get the sentinel key -1 and add nothing.
template <int CTRL>
__device__ __forceinline__ void seg_step(int key, int32_t& ax, int32_t& ay) {
  const int k2 = __builtin_amdgcn_update_dpp(-1, key, CTRL, 0xf, 0xf, false);
  const int x2 = __builtin_amdgcn_update_dpp(0, ax, CTRL, 0xf, 0xf, false);
  const int y2 = __builtin_amdgcn_update_dpp(0, ay, CTRL, 0xf, 0xf, false);
  if (k2 == key) {
    ax += x2;
    ay += y2;
  }
}

// With COM, the workgroups of the first pixel chunk also form each frame's exact integer first
// moments from the same event loads (Eq. 4): a lane folds its four events into runs of equal
// frame, a segmented scan over each row of 16 lanes (events are in frame order) merges the runs
// that cross lanes, and one LDS atomic per run end adds them to the frame's window sums (int32: a window
// holds at most kBinWin events, each |kx - cx| < 2^16), which thread f folds into its frame's
// int64 sums at the next window barrier.  The centre of mass is then S / N_f by one double
// division, as the centre-of-mass kernel computes it.
template <typename DT, bool BOX, bool COM>
__global__ void __launch_bounds__(kBinThreads) k_bin(const int32_t* __restrict__ idx,
                                                     const int64_t* __restrict__ off, int64_t frame0,
                                                     int64_t n_frames, int32_t npix,
                                                     const int16_t* __restrict__ lut,
                                                     const RowRun* __restrict__ rows, BinBox box, int32_t n_k,
                                                     int64_t F, DT* __restrict__ D, ComOut com, GeomOut geo,
                                                     SetsJob sj, int32_t* status) {
  extern __shared__ int16_t s_box[];  // [bh][bw] kept-bin index of each bin of the box, or -1
  __shared__ __align__(16) uint32_t s_hist[kBinWords];
  __shared__ uint32_t s_map[(kBinWin + 16) / 4];
  __shared__ int32_t s_rel[kBinFrames + 1];
  __shared__ int64_t s_base;
  __shared__ int32_t s_mom[COM ? 2 * kBinFrames : 1];  // [x | y][frame] moment sums of a window
  const int t = threadIdx.x;
  const int lane = t & 63;
  if (geo.mark && blockIdx.x == 0 && t == 0) *geo.mark = 0ull;
  if (geo.rows && blockIdx.x == 0) {
    // the counters' LDS is free until the first pass clears it
    build_geometry(box.bin, geo.nbx, geo.nby, geo.cx, geo.cy, geo.r2, geo.rows, geo.kc, (int32_t*)s_hist);
    __syncthreads();
  }
  if constexpr (BOX) {
    // workgroups 1, 2, ... build the interval table and the mask, one word per wave, with Kc of
    // the lane's pixel from the box's row runs (as the geometry computes it)
    const int64_t word = (int64_t)(blockIdx.x - 1) * (kBinThreads / 64) + (t >> 6);
    if (sj.cst && blockIdx.x >= 1 && word < (int64_t)sj.ncs * sj.nmw) {
      const int kd = 64 * (int)(word % sj.nmw) + lane;
      double2 k = make_double2(0.0, 0.0);
      if (kd < sj.n_k) {
        int r = 0;
        while (r < box.bh - 1 && kd >= box.start[r] + box.hi[r] - box.lo[r]) ++r;
        k = make_double2(bin_centre(box.bin, box.lo[r] + kd - box.start[r], geo.cx),
                         bin_centre(box.bin, box.by0 + r, geo.cy));
      }
      sets_word(sj, word, lane, k);
    }
  }
  // workgroups added for the table only (tiny scans) bin nothing
  if ((int64_t)(blockIdx.x / ((n_k + kBinKd - 1) / kBinKd)) * kBinFrames >= n_frames) return;
  const int nchunks = (n_k + kBinKd - 1) / kBinKd;
  const int kd0 = (int)(blockIdx.x % nchunks) * kBinKd;
  const int kc = n_k - kd0 < kBinKd ? n_k - kd0 : kBinKd;
  const int64_t fb = frame0 + (int64_t)(blockIdx.x / nchunks) * kBinFrames;
  const int64_t fend = frame0 + n_frames;
  const int nf = (int)((fend - fb) < kBinFrames ? (fend - fb) : kBinFrames);
  if (!load_rel_offsets(off, fb, nf, s_rel, &s_base, status)) return;
  const bool com_blk = COM && kd0 == 0;  // workgroup-uniform
  if constexpr (COM) {
    if (com_blk)
      for (int i = t; i < 2 * kBinFrames; i += kBinThreads) s_mom[i] = 0;
  }
  int64_t msx = 0, msy = 0;  // thread t: the moments of frame t so far
  // after a barrier that follows a window's atomics and precedes the next window's
  auto fold_moments = [&]() {
    if (COM && com_blk && t < kBinFrames) {
      msx += s_mom[t];
      msy += s_mom[kBinFrames + t];
      s_mom[t] = 0;
      s_mom[kBinFrames + t] = 0;
    }
  };
  if constexpr (BOX) {
    // kept index of each bin of the box from the row runs (the rule of the per-pixel table)
    for (int i = t; i < box.bw * box.bh; i += kBinThreads) {
      const int ry = i / box.bw, bx = box.bx0 + i % box.bw;
      s_box[i] = (int16_t)(bx >= box.lo[ry] && bx < box.hi[ry] ? box.start[ry] + bx - box.lo[ry] : -1);
    }
  }
  __syncthreads();
  const int wide = __syncthreads_or(t < nf && s_rel[t + 1] - s_rel[t] > 255);
  const int span = s_rel[nf];
  const int lo_t = t < nf ? s_rel[t] : 0, hi_t = t < nf ? s_rel[t + 1] : 0;
  const int64_t base = s_base;
  uint8_t* map = (uint8_t*)s_map;
  int32_t bad = 0;
  const int npass = wide ? 2 : 1;
  const int kpp = (kc + npass - 1) / npass;       // pixels per pass
  const int wpr = wide ? kBinFrames / 2 : kBinFrames / 4;  // words per pixel row
  const int wps = wpr + 1;                        // row stride in words (padded)
  const uint32_t cap = sizeof(DT) == 1 ? 255u : 65535u;
  // 8-bit counts go out as 16 frames (four counter words) per 16-byte store when aligned
  const bool vec = sizeof(DT) == 1 && !wide && (((uintptr_t)D & 15) == 0) && (F & 15) == 0 && (fb & 15) == 0;
  for (int pass = 0; pass < npass; ++pass) {
    const int ka = kd0 + pass * kpp;
    const int kn = (kd0 + kc) - ka < kpp ? (kd0 + kc) - ka : kpp;
    for (int i = t; i < (kn * wps + 3) >> 2; i += kBinThreads) ((uint4*)s_hist)[i] = make_uint4(0u, 0u, 0u, 0u);
    for (int w0 = 0; w0 < span; w0 += kBinWin) {
      const int wn = span - w0 < kBinWin ? span - w0 : kBinWin;
      const int64_t a0 = base + w0;
      const int sh = (int)((((uintptr_t)(idx + a0)) & 15) >> 2);  // map[sh + j] <-> event a0 + j
      __syncthreads();
      fold_moments();
      {
        // frame t's events of this window: map entries [lo, hi)
        const int lo = (lo_t > w0 ? lo_t : w0) - w0 + sh;
        const int hi = (hi_t < w0 + wn ? hi_t : w0 + wn) - w0 + sh;
        int j = lo;
        for (; j < hi && (j & 3); ++j) map[j] = (uint8_t)t;
        const uint32_t word = (uint32_t)(t & 0xff) * 0x01010101u;
        for (; j + 4 <= hi; j += 4) s_map[j >> 2] = word;
        for (; j < hi; ++j) map[j] = (uint8_t)t;
      }
      __syncthreads();
      // Positions p = 4 g + q of the 16-byte aligned run from ib: [sh, sh + wn) are this window's
      // events.  Every group g < ng holds at least one of them, so its whole 16-byte line lies in
      // the event array's pages; the other positions of the line are masked out.
      const int32_t* ib = idx + (a0 - sh);
      const int ng = (wn + sh + 3) >> 2;
      constexpr int U = kBinWin / (4 * kBinThreads);  // groups per thread in flight: one pass per window
      for (int g0 = t; g0 < ng; g0 += U * kBinThreads) {
        int4 kv[U];
        uint32_t fr4[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int g = g0 + u * kBinThreads;
          kv[u] = make_int4(0, 0, 0, 0);
          fr4[u] = 0u;
          if (g < ng) {
            kv[u] = *(const int4*)(ib + 4 * g);
            fr4[u] = s_map[g];
          }
        }
        // the table lookups are issued together; masked or out-of-range positions look up pixel 0
        int kd[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int p = 4 * (g0 + u * kBinThreads) + q;
            const int k = q == 0 ? kv[u].x : q == 1 ? kv[u].y : q == 2 ? kv[u].z : kv[u].w;
            const bool ok = (uint32_t)(p - sh) < (uint32_t)wn;
            const bool in = (uint32_t)k < (uint32_t)npix;
            if (ok && !in) bad |= STEM_ERANGE;
            const uint32_t kk = ok && in ? (uint32_t)k : 0u;  // 32-bit offset from the table base
            int v;
            if constexpr (BOX) {
              const uint32_t ky = magic_div(kk, box.mw), kx = kk - ky * (uint32_t)box.W;
              const uint32_t rx = (box.mbin ? __umulhi(kx, box.mbin) : kx) - (uint32_t)box.bx0;
              const uint32_t ry = (box.mbin ? __umulhi(ky, box.mbin) : ky) - (uint32_t)box.by0;
              v = rx < (uint32_t)box.bw && ry < (uint32_t)box.bh ? (int)s_box[ry * box.bw + rx] : -1;
            } else {
              v = (int)*(const int16_t*)((const char*)lut + 2u * kk);
            }
            kd[u][q] = ok && in && v >= 0 ? v - ka : -1;
          }
        if constexpr (COM) {
          if (com_blk && pass == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
              // runs of equal frame among the lane's events in this window; all but the last go
              // to LDS at once (a lane crosses a frame boundary only at frames of few events)
              int fc = -1;
              int32_t ax = 0, ay = 0;
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int p = 4 * (g0 + u * kBinThreads) + q;
                if ((uint32_t)(p - sh) >= (uint32_t)wn) continue;
                const int k = q == 0 ? kv[u].x : q == 1 ? kv[u].y : q == 2 ? kv[u].z : kv[u].w;
                const int f = (int)((fr4[u] >> (8 * q)) & 0xffu);
                if (f != fc) {
                  if (fc >= 0) {
                    atomicAdd(&s_mom[fc], ax);
                    atomicAdd(&s_mom[kBinFrames + fc], ay);
                  }
                  fc = f;
                  ax = ay = 0;
                }
                // an index outside the detector adds nothing (it is reported by the binning)
                if ((uint32_t)k < (uint32_t)npix) {
                  const uint32_t ky = magic_div((uint32_t)k, box.mw), kx = (uint32_t)k - ky * (uint32_t)box.W;
                  ax += (int32_t)kx - com.cx;
                  ay += (int32_t)ky - com.cy;
                }
              }
              // the lanes' last runs: inclusive scan within each row of 16 lanes, segmented by
              // frame, by DPP row shifts (register moves, no LDS traffic); lower lanes hold
              // earlier events, and the lanes of this loop trip are a prefix of the wave
              const int key = fc >= 0 ? fc : 256 + lane;  // a lane without events merges with none
              seg_step<0x111>(key, ax, ay);               // row_shr:1
              seg_step<0x112>(key, ax, ay);               // row_shr:2
              seg_step<0x114>(key, ax, ay);               // row_shr:4
              seg_step<0x118>(key, ax, ay);               // row_shr:8
              // a run ends where the next lane's frame differs, at a row's last lane (row_shl:1
              // leaves the sentinel there) and before a lane outside this loop trip
              const int nkey = __builtin_amdgcn_update_dpp(-2, key, 0x101, 0xf, 0xf, false);
              const bool last = g0 + 1 >= ng || nkey != key;
              if (fc >= 0 && last) {
                atomicAdd(&s_mom[fc], ax);
                atomicAdd(&s_mom[kBinFrames + fc], ay);
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            // a dropped bin (-1), or a pixel of another chunk or pass, is not counted here
            if ((uint32_t)kd[u][q] >= (uint32_t)kn) continue;
            const uint32_t f = (fr4[u] >> (8 * q)) & 0xffu;
            const int shift = wide ? 16 * (f & 1) : 8 * (f & 3);
            const int col = wide ? (f >> 1) : (f >> 2);
            atomicAdd(&s_hist[__umul24(kd[u][q], wps) + col], 1u << shift);
          }
      }
    }
    __syncthreads();
    if (vec) {
      // four counter words (16 frames) of one pixel row per thread and step
      const int qpr = wpr / 4;
      for (int i = t; i < kn * qpr; i += kBinThreads) {
        const int kd = i / qpr, q4 = i % qpr;
        const int f0 = 16 * q4;
        if (f0 >= nf) continue;
        const uint32_t* hw = s_hist + kd * wps + 4 * q4;
        uint8_t* dst = (uint8_t*)D + (int64_t)(ka + kd) * F + (fb + f0);
        if (f0 + 16 <= nf) {
          *(uint4*)dst = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        } else {
          for (int j = 0; f0 + j < nf; ++j) dst[j] = (uint8_t)(hw[j >> 2] >> (8 * (j & 3)));
        }
      }
    } else {
      // one counter word per thread and step: fpw consecutive frames of one pixel row
      const int fpw = wide ? 2 : 4;
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
        for (int j = 0; j < fpw && f0 + j < nf; ++j) {
          if (c[j] > cap) bad |= STEM_EOVERFLOW;
          dst[j] = (DT)c[j];
        }
      }
    }
    __syncthreads();
  }
  if constexpr (COM) {
    fold_moments();  // the pass loop ends with a barrier: the last window's sums
    if (com_blk && t < nf) {
      const int64_t fr = fb + t;
      const int64_t n = hi_t - lo_t;
      const int64_t sx = msx, sy = msy;
      const double x = n > 0 ? (double)sx / (double)n : 0.0;
      const double y = n > 0 ? (double)sy / (double)n : 0.0;
      if (com.com64) {
        com.com64[fr] = x;
        com.com64[com.nplane + fr] = y;
      }
      if (com.com32) {
        com.com32[fr] = (float)x;
        com.com32[com.nplane + fr] = (float)y;
      }
      if (com.counts) com.counts[fr] = (int32_t)n;
    }
  }
  if (bad) report(status, bad);
}

// The kept bins' bounding box and its rows' runs; true when the binning uses the LDS bin table
// over it (and then also takes the geometry's and the interval table's work).
static bool make_box(const stem_det& det, double r2, BinBox& box) {
  const int nbx = det.W / det.bin, nby = det.H / det.bin;
  box = BinBox{};
  int bxa = nbx, bxb = 0, bya = nby, byb = 0;
  int run_start = 0;
  for (int by = 0; by < nby; ++by) {
    int lo, hi;
    kept_run(det.bin, by, nbx, det.cx, det.cy, r2, lo, hi);
    if (hi <= lo) continue;
    bxa = lo < bxa ? lo : bxa;
    bxb = hi > bxb ? hi : bxb;
    if (bya == nby) bya = by;
    byb = by + 1;
    // row runs of the box's rows, in box-row order (kept rows of the box are contiguous)
    if (by - bya < kBoxRows) {
      box.start[by - bya] = run_start;
      box.lo[by - bya] = lo;
      box.hi[by - bya] = hi;
    }
    run_start += hi - lo;
  }
  box.W = det.W;
  box.bin = det.bin;
  box.mw = make_magic((uint32_t)det.W);
  box.mbin = det.bin == 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) + det.bin - 1) / det.bin);
  box.bx0 = bxa;
  box.by0 = bya;
  box.bw = bxb > bxa ? bxb - bxa : 0;
  box.bh = byb > bya ? byb - bya : 0;
  // the LDS table when it is small; the bin divisions by multiply-high are exact for W, H < 2^16
  const int64_t cells = (int64_t)box.bw * box.bh;
  return cells > 0 && cells <= kBinBoxMax && box.bh <= kBoxRows && det.W < 65536 && det.H < 65536;
}

bool bin_builds_sets(const stem_det& det, double r2) {
  BinBox box;
  return make_box(det, r2, box);
}

int launch_bin(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, double r2, RowRun* rows, double2* kc, int16_t* lut, int n_k, int64_t F,
               void* D, int d_bits, int32_t* status, hipStream_t stream, const ComOut* com, const SetsJob* sets,
               unsigned long long* mark) {
  if (n_frames == 0) return STEM_OK;
  const int nchunks = (n_k + kBinKd - 1) / kBinKd;
  const int64_t fblocks = (n_frames + kBinFrames - 1) / kBinFrames;
  const int nbx = det.W / det.bin, nby = det.H / det.bin;
  BinBox box;
  const bool use_box = make_box(det, r2, box);
  const int64_t cells = (int64_t)box.bw * box.bh;
  const size_t lds = use_box ? (size_t)((cells * 2 + 15) & ~15ll) : 0;
  // BOX with the interval table: enough workgroups for one wave per mask word besides the first
  const SetsJob sj = use_box && sets ? *sets : SetsJob{};
  int64_t blocks = fblocks * nchunks;
  if (sj.cst) {
    const int64_t need = 1 + ((int64_t)sj.ncs * sj.nmw + kBinThreads / 64 - 1) / (kBinThreads / 64);
    if (need > blocks) blocks = need;
  }
  const dim3 grid((unsigned)blocks);
  // BOX: the binning kernel's first workgroup writes the row runs and bin centres; otherwise the
  // per-pixel table needs them first
  GeomOut geo{};
  if (use_box) {
    geo = GeomOut{rows, kc, nbx, nby, det.cx, det.cy, r2, nullptr};
  } else {
    if (int st = launch_geometry(det, r2, rows, kc, stream)) return st;
    // the per-pixel table, read by the binning kernel
    STEM_TRACE("pixel_lut", stream);
    const int64_t npix = (int64_t)det.W * det.H;
    hipLaunchKernelGGL(k_pixel_lut, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, stream, rows, det.W, det.H,
                       det.bin, lut);
    STEM_LAUNCH_CHECK();
  }
  geo.mark = mark;
  STEM_TRACE(com ? "bin_com" : "bin_densify", stream);
  const ComOut co = com ? *com : ComOut{};
  const int npix = det.W * det.H;
  auto go = [&](auto dt, auto bx, auto cm) {
    using DT = decltype(dt);
    constexpr bool BX = decltype(bx)::value, CM = decltype(cm)::value;
    hipLaunchKernelGGL((k_bin<DT, BX, CM>), grid, dim3(kBinThreads), BX ? lds : 0, stream, idx, off, frame0,
                       n_frames, npix, lut, rows, box, n_k, F, (DT*)D, co, geo, sj, status);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  if (d_bits == 8) {
    if (use_box) com ? go(uint8_t{}, T_{}, T_{}) : go(uint8_t{}, T_{}, F_{});
    else com ? go(uint8_t{}, F_{}, T_{}) : go(uint8_t{}, F_{}, F_{});
  } else {
    if (use_box) com ? go(uint16_t{}, T_{}, T_{}) : go(uint16_t{}, T_{}, F_{});
    else com ? go(uint16_t{}, F_{}, T_{}) : go(uint16_t{}, F_{}, F_{});
  }
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

extern "C" int virtual_annular(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                               const stem_det* det, const stem_scan* scan, int n_det, const double* h_r_in,
                               const double* h_r_out, int32_t* d_out, int32_t* d_status, void* stream_) {
  if (!d_idx || !d_off || !det || !scan || !d_out || !h_r_in || !h_r_out) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  if (scan->ny <= 0 || scan->nx <= 0 || n_det < 1 || n_det > STEM_MAX_ANNULI) return STEM_EINVAL;
  const int64_t F = (int64_t)scan->ny * scan->nx;
  if (frame0 < 0 || n_frames < 0 || frame0 + n_frames > F) return STEM_EINVAL;
  Annuli an;
  const double big = 9.0e18;  // beyond every squared distance of a detector with W*H < 2^31
  for (int j = 0; j < STEM_MAX_ANNULI; ++j) {
    an.lo[j] = an.hi[j] = 0;
    if (j >= n_det) continue;
    const double a = h_r_in[j], b = h_r_out[j];
    if (!(a >= 0.0) || !(b >= 0.0)) return STEM_EINVAL;  // also rejects NaN
    // d2 >= a^2 and d2 < b^2 for an integer d2  <=>  d2 >= ceil(a^2) and d2 < ceil(b^2)
    const double a2 = std::ceil(a * a), b2 = std::ceil(b * b);
    an.lo[j] = a2 >= big ? (int64_t)big : (int64_t)a2;
    an.hi[j] = b2 >= big ? (int64_t)big : (int64_t)b2;
  }
  if (n_frames == 0) return STEM_OK;
  hipStream_t s = (hipStream_t)stream_;
  const int64_t blocks = (n_frames + kComFrames - 1) / kComFrames;
  const Magic mw = make_magic((uint32_t)det->W);
  STEM_TRACE("virtual_annular", s);
  const dim3 grid((unsigned)blocks), blk(kComThreads);
  const int npix = det->W * det->H;
  if (n_det <= 1)
    hipLaunchKernelGGL(k_annular<1>, grid, blk, 0, s, d_idx, d_off, frame0, n_frames, mw, det->cx, det->cy, npix, an,
                       F, d_out, d_status);
  else if (n_det <= 2)
    hipLaunchKernelGGL(k_annular<2>, grid, blk, 0, s, d_idx, d_off, frame0, n_frames, mw, det->cx, det->cy, npix, an,
                       F, d_out, d_status);
  else if (n_det <= 4)
    hipLaunchKernelGGL(k_annular<4>, grid, blk, 0, s, d_idx, d_off, frame0, n_frames, mw, det->cx, det->cy, npix, an,
                       F, d_out, d_status);
  else if (n_det <= 8)
    hipLaunchKernelGGL(k_annular<8>, grid, blk, 0, s, d_idx, d_off, frame0, n_frames, mw, det->cx, det->cy, npix, an,
                       F, d_out, d_status);
  else
    hipLaunchKernelGGL(k_annular<16>, grid, blk, 0, s, d_idx, d_off, frame0, n_frames, mw, det->cx, det->cy, npix,
                       an, F, d_out, d_status);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}

extern "C" int sum_frames(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                          const stem_det* det, uint32_t* d_sum, float* d_mean, int32_t* d_status, void* stream_) {
  if (!d_idx || !d_off || !det || !d_sum || frame0 < 0 || n_frames <= 0) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  hipStream_t s = (hipStream_t)stream_;
  const int W = det->W, H = det->H;
  const int bw = W < kSumBox ? W : kSumBox, bh = H < kSumBox ? H : kSumBox;
  int bx0 = det->cx - bw / 2, by0 = det->cy - bh / 2;
  bx0 = bx0 < 0 ? 0 : (bx0 > W - bw ? W - bw : bx0);
  by0 = by0 < 0 ? 0 : (by0 > H - bh ? H - bh : by0);
  {
    STEM_TRACE("sum_frames", s);
    hipLaunchKernelGGL(k_sum_events, dim3(kSumBlocks), dim3(256), 0, s, d_idx, d_off, frame0, n_frames,
                       make_magic((uint32_t)W), W * H, bx0, by0, bw, bh, d_sum, d_status);
    STEM_LAUNCH_CHECK();
  }
  if (d_mean) {
    const int64_t npix = (int64_t)W * H;
    hipLaunchKernelGGL(k_frame_mean, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, d_sum, npix,
                       (double)n_frames, d_mean);
    STEM_LAUNCH_CHECK();
  }
  return STEM_OK;
}

extern "C" int eer_decode_rle(const int32_t* d_dist, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                              const stem_det* det, int32_t* d_idx, int32_t* d_status, void* stream_) {
  if (!d_dist || !d_off || !det || !d_idx || frame0 < 0 || n_frames < 0) return STEM_EINVAL;
  if (det->W <= 0 || det->H <= 0 || (int64_t)det->W * det->H >= (1ll << 31)) return STEM_EINVAL;
  if (n_frames == 0) return STEM_OK;
  hipStream_t s = (hipStream_t)stream_;
  const int64_t blocks = (n_frames + kComFrames - 1) / kComFrames;
  STEM_TRACE("decode_rle", s);
  hipLaunchKernelGGL(k_decode_rle, dim3((unsigned)blocks), dim3(kComThreads), 0, s, d_dist, d_off, frame0, n_frames,
                     det->W * det->H, d_idx, d_status);
  STEM_LAUNCH_CHECK();
  return STEM_OK;
}
