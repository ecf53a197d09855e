// Internal launchers shared between the translation units of the stem4d library.
#pragma once

#include "common.h"
#include "geom.h"
#include "optics.h"

namespace stem {

// ---- eer.hip ---------------------------------------------------------------------------------
int launch_com(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, int64_t nplane, double* com64, float* com32, int32_t* counts,
               int32_t* status, hipStream_t stream);
// kept-set geometry: row runs and bin centres Kc
int launch_geometry(const stem_det& det, double r2, RowRun* rows, double2* kc, hipStream_t stream);
// centre-of-mass outputs formed by the binning pass itself ([2][nplane] planes, each may be null)
struct ComOut {
  double* com64;
  float* com32;
  int32_t* counts;
  int64_t nplane;
  int32_t cx, cy;
};
// binning; also writes the kept-set geometry (row runs, bin centres Kc), and builds the per-pixel
// table lut[W*H] first when the kept bins' box is too large for LDS.  With com, the same pass also
// writes the frames' centre of mass (as launch_com does).
// With sets (and the LDS bin table: bin_builds_sets), the binning also builds the interval table
// and the active-pixel mask of the fused column sum.  With mark, its first thread clears that word
// (the state's FINALIZE mark, at an accumulation from frame 0).
int launch_bin(const int32_t* idx, const int64_t* off, int64_t frame0, int64_t n_frames,
               const stem_det& det, double r2, RowRun* rows, double2* kc, int16_t* lut, int n_k, int64_t F,
               void* D, int d_bits, int32_t* status, hipStream_t stream, const ComOut* com = nullptr,
               const SetsJob* sets = nullptr, unsigned long long* mark = nullptr);
bool bin_builds_sets(const stem_det& det, double r2);

// ---- fft2.hip: batched row FFTs of length n (power of two, 32..1024) --------------------------
enum RowIn { IN_C64 = 0, IN_C64_SUM = 1, IN_F32_PAIR = 2, IN_F64_PAIR = 3, IN_HALF_C64 = 4, IN_U8 = 5, IN_U16 = 6 };
enum RowOut { OUT_T_C64 = 0, OUT_ROW_C64 = 1, OUT_ROW_RE = 2, OUT_ROW_IM = 3, OUT_T_RE = 4, OUT_T_IM = 5, OUT_X = 6 };

struct RowFftArgs {
  int64_t nrows;
  // inputs
  const float2* in_c;      // IN_C64 / IN_C64_SUM: row r at in_c + r*n (+ p*part_stride);
                           // IN_HALF_C64: entries 0..n/2 of a Hermitian row at in_c + r*(n/2+1)
  int64_t part_stride;
  int32_t nparts;
  const int64_t* part_seg; // IN_C64_SUM: if set, row r adds rows part_seg[r] .. part_seg[r+1]-1 of in_c
                           // (n values each) instead of the nparts planes, clamped to
  int64_t part_seg_rows;   // the rows in_c holds
  float2* sum_out;         // IN_C64_SUM: if set, the summed input is also stored here (row-major)
  const float* in_f0;      // IN_F32_PAIR: re = in_f0[r*n + j]*s0, im = in_f1[...]*s1 (in_f1 may be null)
  const float* in_f1;
  const double* in_d0;     // IN_F64_PAIR
  const double* in_d1;
  const void* in_u;        // IN_U8 / IN_U16 (generic lengths only): real row r at in_u + r*n
  float s0, s1;
  // outputs
  float2* out_c;           // OUT_T_*: element (r, m) at out[m*out_stride + r]; OUT_ROW_*: out[r*n + m];
                           // OUT_X (generic lengths only): m <= n/2 of row r = kd*xrows + y at
                           // out[(kd*(n/2+1) + m)*xrows + y]
  int32_t xrows;
  float* out_f;
  int64_t out_stride;
  float2 osc;              // complex factor applied to every output value
  const char* tag;         // name under which the launch is traced
  // IN_C64_SUM: if norm_cnt is set, every summed element (r, n) is divided by norm_cnt[r*n + n]
  // (0 where that count is 0)
  const int32_t* norm_cnt;
  // IN_C64_SUM: if stats is set, workgroup 0 also writes stats[0] = the sum of the pair counts
  // (low 40 bits of wcnt[0, nwcnt)), stats[1] = stats_groups, stats[2] = 8 x the sum of the loads
  // (wcnt >> 40), stats[3] = stats_chunks
  const unsigned long long* wcnt;
  int64_t nwcnt;
  unsigned long long* stats;
  int32_t stats_groups;
  int32_t stats_chunks;
  unsigned long long* ready_out;  // IN_C64_SUM with stats: if set, the first workgroup also stores
  unsigned long long ready_val;   // ready_val there (the state's mark of a finished FINALIZE)
};

int launch_row_fft(int n, bool inverse, RowIn in, RowOut out, const RowFftArgs& a, hipStream_t stream);

// lengths the wavefront FFT takes (powers of two in [32, 1024]); the others go to the generic FFT
inline bool fast_length(int n) { return is_pow2_in(n, 32, 1024); }
// lengths the library transforms: the fast ones, and even N = 2^a 3^b 5^c in [16, 4096]
bool scan_length_ok(int n);

// ---- ssb.hip ---------------------------------------------------------------------------------
size_t ssb_layout(const stem_det& det, const stem_scan& scan, const stem_optics& optics,
                  const stem_ssb& ssb, int n_k, struct SsbLayout* lay);

}  // namespace stem
