/*
 * stem4d.h -- C ABI of the MI355X (gfx950) event-based 4D-STEM phase-contrast library.
 *
 * The library turns linear-index electron-event lists (Fig. 1b and Sec. II of Pelz et al.,
 * "Real-time interactive 4D-STEM phase-contrast imaging from electron event representation
 * data") into a centre-of-mass DPC phase image (Sec. V) and a single-sideband ptychographic
 * phase image (Sec. IV), plus the adjoint of the sideband phase.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Events: a dataset is a CSR pair.  idx[C] (int32) holds one linear detector index
 *    k = ky*W + kx per electron; off[F+1] (int64) holds frame boundaries, frame f owning
 *    idx[off[f] .. off[f+1]).  Frames are probe positions in raster order f = ry*Nx + rx.
 *    Events inside a frame may come in any order and may repeat.
 *  - Memory: the caller owns every buffer.  Pointers named d_* are device pointers on the
 *    current HIP device, h_* are host pointers.  Nothing is allocated inside the calls.
 *  - Streams: `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue work
 *    and return; outputs are valid once the stream has been synchronised.
 *  - Errors: every call returns a stem_status.  Argument errors that the host can see are
 *    returned at once and nothing is enqueued.  Errors that depend on the data (an index
 *    outside the detector, non-monotone offsets, a count that does not fit its type) are
 *    found on the device and OR-ed as status bits into the caller's int32 *d_status, which
 *    the caller reads after synchronising (d_status may be NULL to skip those checks'
 *    reporting; the kernels still never read or write out of bounds).
 *  - Re-entrancy: calls on distinct workspaces may run concurrently; calls sharing a
 *    workspace must be ordered on one stream.
 *  - Units: detector coordinates are unbinned pixels relative to the zero-frequency pixel
 *    (cx, cy); dk is the detector pixel size in 1/angstrom; step is the scan step in
 *    angstrom; lam the electron wavelength in angstrom; aberration coefficients in angstrom.
 */
#ifndef STEM4D_H
#define STEM4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------------------------------- */
/* Status codes.  Host-returned codes are single values; device-side codes are bits OR-ed   */
/* into *d_status.                                                                          */

typedef enum {
  STEM_OK = 0,
  STEM_EINVAL = 1,      /* bad argument (NULL pointer, size, geometry, unsupported shape)   */
  STEM_ERANGE = 2,      /* device: an event index is < 0 or >= W*H                          */
  STEM_EOFFSETS = 4,    /* device: offsets decrease, or do not bound the chunk's events     */
  STEM_EOVERFLOW = 8,   /* device: a binned count does not fit the binned-cube element type */
  STEM_EWORKSPACE = 16, /* workspace / state buffer smaller than the size query returns     */
  STEM_EHIP = 32,       /* a HIP runtime call failed (launch, copy)                         */
  STEM_ESTATE = 64      /* device: the state holds no FINALIZE (a REFOCUS or backward call)  */
} stem_status;

const char* stem_strerror(int status);

/* Library version as 10000*major + 100*minor + patch. */
int stem_version(void);

/* ---------------------------------------------------------------------------------------- */
/* Parameters                                                                               */

/* Detector.  W, H unbinned pixels (W*H < 2^31); (cx, cy) the zero-frequency pixel
 * (usually (W/2, H/2)); bin the binning factor of the sideband path, dividing W and H. */
typedef struct {
  int32_t W, H;
  int32_t cx, cy;
  int32_t bin;
} stem_det;

/* Scan grid: Ny x Nx probe positions, spacing `step` angstrom.  The transforms take Ny and Nx
 * of the form 2^a 3^b 5^c, even, in [16, 4096] (the fused single-wave kernels serve powers of
 * two in [32, 1024]; the other lengths run a mixed-radix LDS FFT and separate sum kernels);
 * centre of mass alone takes any size. */
typedef struct {
  int32_t ny, nx;
  double step;
} stem_scan;

/* Probe optics: wavelength lam, bright-field disk radius r_bf (unbinned pixels; the disk
 * radius alpha/lambda of Sec. IV expressed in pixels), detector pixel size dk (1/angstrom)
 * and aberration coefficients c[8] = (C1, A1a, A1b, B2a, B2b, A2a, A2b, C3) of
 * chi = (2 pi/lam) [C1 w^2/2 + A1a (wx^2-wy^2)/2 + A1b wx wy + B2a w^2 wx/3 + B2b w^2 wy/3
 *                   + A2a (wx^3 - 3 wx wy^2)/3 + A2b (3 wx^2 wy - wy^3)/3 + C3 w^4/4],
 * w = lam * k. */
typedef struct {
  double lam;
  double r_bf;
  double dk;
  double c[8];
} stem_optics;

/* DPC integration (Sec. V): step size mu (0.5 in the paper), low-pass lam1, high-pass
 * lam2 regularisers, number of gradient-descent iterations n_iter (>= 0). */
typedef struct {
  double mu, lam1, lam2;
  int32_t n_iter;
} stem_dpc;

enum { STEM_FFT_FP32 = 0, STEM_DFT_BF16_SPLIT = 1, STEM_DFT_FP16_SPLIT = 2 };
enum { STEM_G_RECOMPUTE = 0, STEM_G_STORE = 1 };

/* Sideband path options.
 *  precision:   STEM_FFT_FP32 (FP32 FFT) or one of the split-precision MFMA scan DFTs.
 *  normalize:   0 = plain Eq. 3 sum; 1 = divide T(Q) by the number of pixels in the set.
 *  g_mode:      STEM_G_STORE keeps the row-transformed cube of every pixel (written during
 *               ACCUMULATE) and, from FINALIZE on, G(K,Q) on the double-overlap pairs only (the
 *               values Eq. 3 uses): REFOCUS and the adjoint read those.  STEM_G_RECOMPUTE keeps
 *               only the binned counts: every sum and the adjoint transform a chunk of pixels at a
 *               time in a bounded scratch, so the state is a fraction of the STORE one.
 *  d_bits:      8 or 16, element width of the binned count cube (a larger count sets
 *               STEM_EOVERFLOW; it is never clamped silently).
 *  scratch_mib: STEM_G_RECOMPUTE: at most this many MiB of row-transformed columns are held at
 *               once (0: 64 MiB; at least one pixel's); ignored by STEM_G_STORE. */
typedef struct {
  int32_t precision;
  int32_t normalize;
  int32_t g_mode;
  int32_t d_bits;
  int32_t scratch_mib;
} stem_ssb;

/* ---------------------------------------------------------------------------------------- */
/* a1. Event ingest (Sec. IV: the events are loaded directly onto the GPU)                  */

/* Copy a chunk of frames [frame0, frame0 + n_frames) to the device and validate it.
 * h_off[0 .. n_frames] are the chunk's offsets in global event numbering (h_off[0] is the
 * global index of the chunk's first event, h_off[n_frames] - h_off[0] == n_events); they
 * land in d_off[frame0 .. frame0 + n_frames].  h_idx[0 .. n_events) lands in
 * d_idx[h_off[0] .. h_off[0] + n_events).  With h_idx == NULL and h_off == NULL the data is
 * already on the device and is only validated; n_events is then the number of entries of
 * d_idx, and the chunk's events d_off[frame0] .. d_off[frame0 + n_frames] must lie inside
 * [0, n_events).  Host memory should be pinned for the copies to overlap compute.
 * Device checks: offsets non-decreasing and inside the event array (STEM_EOFFSETS; such
 * offsets are never followed), 0 <= idx < W*H (STEM_ERANGE).
 * com_dpc and ssb_reconstruct trust the offsets of the frames they are given: run them only
 * on chunks whose validation reported no STEM_EOFFSETS (event indices outside the detector
 * are skipped there and reported as STEM_ERANGE).
 * Errors: STEM_EINVAL for NULL device pointers, negative sizes, W*H >= 2^31, or host offsets
 * inconsistent with n_events. */
int eer_load_csr(const int32_t* h_idx, const int64_t* h_off, int64_t frame0, int64_t n_frames,
                 int64_t n_events, const stem_det* det, int32_t* d_idx, int64_t* d_off,
                 int32_t* d_status, void* stream);

/* Re-coding of the run-length form (Fig. 1c; Table 1: O(C)) into linear indices: within each
 * frame f of [frame0, frame0 + n_frames), events in ascending pixel order are stored as
 * distances d_0 = k_0, d_i = k_i - k_(i-1) (>= 0; a repeated pixel gives 0), with the same CSR
 * offsets d_off as the linear-index form.  Writes d_idx[e] = sum of the frame's distances up to
 * and including e (a prefix sum restarted at every frame) for the events of those frames.
 * d_dist and d_idx may not overlap.  Indices outside [0, W*H) (from a negative distance or a
 * sum past the detector) are written as -1 and set STEM_ERANGE in d_status.
 * Errors: STEM_EINVAL (NULL pointers, negative frame0 or n_frames, W*H >= 2^31). */
int eer_decode_rle(const int32_t* d_dist, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                   const stem_det* det, int32_t* d_idx, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------------------- */
/* a2 + a3. Centre of mass (Eq. 4, Table 1) and DPC integration (Sec. V)                     */

/* Bytes of workspace com_dpc needs for the integration on this scan grid. */
size_t com_dpc_workspace_bytes(const stem_scan* scan);

/* Centre of mass of frames [frame0, frame0 + n_frames): N_f, Sx = sum(kx - cx),
 * Sy = sum(ky - cy) as exact integers, then COM = S / N_f by one IEEE double division
 * (0 for an empty frame).  Outputs are [2][F] planes (x first, then y) indexed by the
 * global frame number, F = ny*nx; d_com64 and/or d_com32 (the FP32 value is the rounded
 * double) and d_counts[F] may each be NULL.  COM is in unbinned pixels relative to (cx, cy)
 * and uses the full-resolution events (det.bin is ignored).
 * If d_phase != NULL the DPC integration then runs over the whole scan grid (all frames
 * must have been processed by earlier or this call) from d_com64 if given, else d_com32:
 * g = 2 pi dk COM (rad/angstrom), Phi <- Phi + mu conj(D)(Ghat - D Phi)/(lam1 + |2 pi q|^2 +
 * lam2 |2 pi q|^4), D = 2 pi i q, Phi_0 = 0, q = 0 and Nyquist terms held at zero;
 * d_phase[F] = Re IFFT2(Phi) in row-major (ry, rx) order.  ws must hold
 * com_dpc_workspace_bytes(scan) bytes (256-byte aligned) when d_phase != NULL.
 * Errors: STEM_EINVAL (NULL idx/off, no COM output when integrating, frame range outside
 * [0, F), a scan length the transforms do not take when integrating), STEM_EWORKSPACE. */
int com_dpc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
            const stem_det* det, const stem_scan* scan, const stem_optics* optics,
            const stem_dpc* dpc, double* d_com64, float* d_com32, int32_t* d_counts,
            float* d_phase, void* ws, size_t ws_bytes, int32_t* d_status, void* stream);

/* Allocation-free variant of com_dpc, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * computation and outputs as com_dpc without (ws, ws_bytes): the DPC integration's workspace is a
 * library-owned device array of com_dpc_noalloc_max_workspace() bytes (16 MiB, enough for scans
 * with com_dpc_workspace_bytes(scan) up to that size, e.g. 1024 x 1024).  Each GPU the library
 * runs on holds its own copy of the array from the first call there until the process ends.
 * Every call on one GPU shares that copy, so calls that overlap on one GPU (several streams or
 * threads) race: the caller orders them.  Nothing is allocated; nothing needs clearing (every
 * call writes the workspace before reading it).
 * Errors: as com_dpc; STEM_EWORKSPACE when the scan needs more workspace than the maximum;
 * STEM_EHIP if the array's address on the current device cannot be found. */
int com_dpc_noalloc(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                    const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                    const stem_dpc* dpc, double* d_com64, float* d_com32, int32_t* d_counts,
                    float* d_phase, int32_t* d_status, void* stream);

/* Bytes of the device array com_dpc_noalloc uses as its workspace. */
size_t com_dpc_noalloc_max_workspace(void);

/* ---------------------------------------------------------------------------------------- */
/* Virtual detectors from events (Table 1: radial sum, sum of all frames; Sec. III)          */

#define STEM_MAX_ANNULI 16

/* Virtual annular detectors (radial sums).  For each of n_det annuli j (1 <= n_det <=
 * STEM_MAX_ANNULI) and each frame f in [frame0, frame0 + n_frames):
 *   d_out[j*F + f] = number of events of f at a pixel with
 *                    r_in[j]^2 <= (kx - cx)^2 + (ky - cy)^2 < r_out[j]^2
 * in unbinned detector pixels (det.bin is ignored), an exact integer test (the radii are
 * squared in double on the host).  F = scan.ny * scan.nx; d_out is int32 [n_det][F], indexed by
 * the global frame number, written only for the given frames.  h_r_in / h_r_out are host
 * arrays of n_det radii.  One pass over the events: O(C), against O((r_out^2 - r_in^2) F) for
 * dense frames.
 * Errors: STEM_EINVAL (NULL pointers, n_det outside [1, STEM_MAX_ANNULI], a negative or NaN
 * radius, frame range outside [0, F)); STEM_ERANGE / STEM_EOVERFLOW via d_status. */
int virtual_annular(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                    const stem_det* det, const stem_scan* scan, int n_det, const double* h_r_in,
                    const double* h_r_out, int32_t* d_out, int32_t* d_status, void* stream);

/* Sum of the frames [frame0, frame0 + n_frames) (Table 1 "sum all frames"): the
 * position-averaged diffraction pattern (PACBED), or over frames in vacuum the average probe.
 *   d_sum[ky*W + kx] += number of events of those frames at pixel (kx, ky)   (uint32 [H][W])
 * The sum is accumulated (the caller zeroes d_sum once, so chunks can be added). If d_mean is
 * not NULL it then receives d_mean[k] = (float)((double)d_sum[k] / n_frames) (float [H][W]).
 * Only the events [off[frame0], off[frame0 + n_frames]) are read (offsets validated by
 * eer_load_csr).  Asynchronous: the event range is read on the device.
 * Errors: STEM_EINVAL (NULL pointers, n_frames <= 0, negative frame0); via d_status
 * STEM_ERANGE for indices outside [0, W*H) (skipped) and STEM_EOFFSETS for a decreasing range. */
int sum_frames(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
               const stem_det* det, uint32_t* d_sum, float* d_mean, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------------------- */
/* a4 - a7. Single-sideband reconstruction (Sec. IV, Eq. 2, the double-overlap set, Eq. 3)  */

enum {
  STEM_SSB_ACCUMULATE = 0, /* bin a chunk of whole scan rows and row-transform it           */
  STEM_SSB_FINALIZE = 1,   /* column transform, double-overlap sum, phase image             */
  STEM_SSB_REFOCUS = 2,    /* sum again from the stored G with new optics.c / theta         */
  STEM_SSB_ONESHOT = 3     /* ACCUMULATE over all frames, then FINALIZE                      */
};

/* Number of kept binned pixels n_K (bin centres strictly inside the bright-field disk),
 * or a negative stem_status.  Host only. */
int ssb_num_pixels(const stem_det* det, const stem_optics* optics);

/* Bytes of state buffer the sideband path needs.  0 on invalid arguments. */
size_t ssb_state_bytes(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                       const stem_ssb* ssb);

/* Kept pixel k (raster order of bins (bx, by) whose centre
 * Kc = (bin*bx + (bin-1)/2 - cx, bin*by + (bin-1)/2 - cy) satisfies |Kc|^2 < r_bf^2) is
 * binned from the events: D[kd][f] counts the events of frame f in bin kd.  The scan
 * transform G(kd, Q) is the unnormalised 2D DFT of D[kd] over (ry, rx) with
 * exp(-2 pi i Q.R).  For every scan frequency index (my, mx) (numpy fftfreq order,
 * Q = (mx*sx, my*sy) pixels, s = 1/((N*step)*dk)):
 *   T(Q) = sum over kd with |Kc|^2 < r^2, |Kc-Q|^2 < r^2, |Kc+Q|^2 >= r^2 of
 *          G(kd, Q) exp(i (chi(Kc-Q) - chi(Kc) - theta[kd])),
 * distances evaluated in IEEE double without fused operations; T(0) = 0.  With
 * normalize = 1, T(Q) is divided by the number of pixels in the set.  The phase image is
 * phi = Im IFFT2(T) (1/(Ny Nx) normalisation).
 *
 * mode ACCUMULATE: frames [frame0, frame0 + n_frames) must be whole scan rows; bins them
 *   and transforms them along x into the state.  d_phase, d_T unused.
 * mode FINALIZE: needs every row accumulated; writes d_phase[F] (row-major, may be NULL)
 *   and d_T[2F] (interleaved complex64 row-major [my][mx], may be NULL).
 * mode REFOCUS: needs a FINALIZE on this state (with this layout: same det, scan, optics
 *   r_bf/dk/lam and ssb) after its last ACCUMULATE from frame 0 (which voids an earlier
 *   FINALIZE), else its sum reads nothing of the state and reports the device bit
 *   STEM_ESTATE, and d_phase, d_T are undefined; the sum and the phase again for the given
 *   optics.c and theta: from the stored double-overlap values of G (STEM_G_STORE, the paper's
 *   interactive mode), or with G recomputed from the binned counts (STEM_G_RECOMPUTE).
 * mode ONESHOT: ACCUMULATE of all F frames then FINALIZE.
 * d_theta[n_K] (FP32, may be NULL = 0) is the per-pixel probe phase.  det, scan, optics
 * r_bf/dk/lam and ssb must stay the same across the calls sharing a state.
 * Errors: STEM_EINVAL (geometry, sizes, non-row chunks, a scan length the transforms do not
 * take, a split precision with a length other than a power of two in [32, 1024], n_K = 0 or
 * > 4096), STEM_EWORKSPACE; device bits ERANGE/EOVERFLOW, and STEM_ESTATE (REFOCUS). */
int ssb_reconstruct(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                    const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                    const stem_ssb* ssb, int mode, const float* d_theta, void* state,
                    size_t state_bytes, float* d_phase, float* d_T, int32_t* d_status,
                    void* stream);

/* a1 + a2 + a4 in one pass over the events (Eq. 4 beside the binning of Sec. IV):
 * ssb_reconstruct in mode ACCUMULATE or ONESHOT that also writes the centre of mass of frames
 * [frame0, frame0 + n_frames) (all F frames for ONESHOT) exactly as com_dpc does: d_com64 /
 * d_com32 [2][F] planes (x then y, global frame number) and d_counts[F], each may be NULL but
 * not all three; the values are bit-identical to com_dpc's.  The DPC integration can then run
 * from d_com64 (or d_com32) by com_dpc with n_frames = 0.  Same ownership, stream order and
 * error rules as ssb_reconstruct; also STEM_EINVAL for another mode, no COM output, or a
 * detector of 65536 or more pixels in either dimension. */
int ssb_reconstruct_com(const int32_t* d_idx, const int64_t* d_off, int64_t frame0, int64_t n_frames,
                        const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                        const stem_ssb* ssb, int mode, const float* d_theta, void* state,
                        size_t state_bytes, float* d_phase, float* d_T, double* d_com64,
                        float* d_com32, int32_t* d_counts, int32_t* d_status, void* stream);

/* Regions of the state buffer a caller may read after the calls that fill them.
 *  STEM_REGION_D     binned counts D[kd][ry][rx], uint8 or uint16 (d_bits), after ACCUMULATE.
 *  STEM_REGION_X     complex64 [kd][mx][ry], mx in [0, Nx/2]: STEM_G_STORE, after ACCUMULATE, the
 *                    row transform of every pixel (the DFT along rx of D); STEM_G_RECOMPUTE, the
 *                    scratch of the last chunk of pixels (contents unspecified).
 *  STEM_REGION_T     complex64 T(Q) of the last sum, column-major [mx][my].
 *  STEM_REGION_KC    double2 Kc[kd] (x, y) bin centres in unbinned pixels, after ACCUMULATE.
 *  STEM_REGION_STATS uint64 [4] about the last sum (FINALIZE / REFOCUS): [0] number of (pixel, Q)
 *                    pairs in the double-overlap sets; [1] number of partial sums of T combined
 *                    (pixel groups of the fused column kernels; after a REFOCUS from the stored
 *                    values, the pieces that sum was cut into, all columns); [2] bytes of row-transformed
 *                    columns or stored G values the sum kernels read; [3] pixel chunks.
 *  STEM_REGION_PG    STEM_G_STORE, after FINALIZE: G on the double-overlap pairs, complex64.  For
 *                    scan-frequency column mx in [0, Nx) and pixel kd the values G(kd, (my, mx)),
 *                    my over the set in ascending signed frequency, start at entry
 *                    POFF[mx*n_K + kd] (column-major); the region holds an upper bound of entries.
 *  STEM_REGION_POFF  STEM_G_STORE, after FINALIZE: int64 [Nx*n_K + 1] those offsets, the last
 *                    entry the number of pairs.
 *  STEM_REGION_NPAIR int32 [F] number of pixels in the double-overlap set of each Q, column-major
 *                    [mx][my], after a FINALIZE with normalize = 1.
 * Writes the byte offset and size of the region; STEM_EINVAL for bad arguments. */
enum {
  STEM_REGION_D = 0,
  STEM_REGION_X = 1,
  STEM_REGION_T = 2,
  STEM_REGION_KC = 3,
  STEM_REGION_STATS = 4,
  STEM_REGION_PG = 5,
  STEM_REGION_POFF = 6,
  STEM_REGION_NPAIR = 7
};
int ssb_state_region(const stem_det* det, const stem_scan* scan, const stem_optics* optics,
                     const stem_ssb* ssb, int region, size_t* offset, size_t* bytes);

#define STEM_MAX_PANEL 64

/* The scan transform at selected scan frequencies as binned detector images (Fig. 2 shows
 * such a panel of G at fixed Q, the regions where the sidebands overlap the bright-field
 * disk).  For j < n_q (1 <= n_q <= STEM_MAX_PANEL), Q_j = (h_my[j], h_mx[j]) frequency indices
 * in numpy fftfreq order (0 <= my < Ny, 0 <= mx < Nx), and every bin (bx, by) of the binned
 * detector (nbx = W/bin, nby = H/bin):
 *   d_img[(j*nby + by)*nbx + bx] = G(kd, Q_j) for the kept bin kd at (bx, by), 0 for a dropped bin
 * as complex64 (interleaved re, im).  The state must hold a finished reconstruction with these
 * arguments (ACCUMULATE of every row at least): G is computed with FP64 accumulation as the DFT
 * along ry of the row-transformed cube (g_mode STORE; for mx > Nx/2 as conj G(kd, -Q), D being
 * real) or as the 2D DFT of the binned counts (g_mode RECOMPUTE).
 * Errors: STEM_EINVAL (NULL pointers, n_q outside [1, STEM_MAX_PANEL], an index outside its
 * range), STEM_EWORKSPACE. */
int ssb_g_panel(const stem_det* det, const stem_scan* scan, const stem_optics* optics, const stem_ssb* ssb,
                const void* state, size_t state_bytes, int n_q, const int32_t* h_my, const int32_t* h_mx,
                float* d_img, void* stream);

/* ---------------------------------------------------------------------------------------- */
/* a8. Adjoint of the sideband phase (not in the paper)                                     */

/* Given gbar = dL/dphi (d_dLdphi[F], FP32 row-major) for the phase of the last FINALIZE or
 * REFOCUS on this state (same optics, theta), accumulates
 *   Tbar = (i/N_R) FFT2(gbar),  w = Re(conj(Tbar(Q)) i G(kd,Q) exp(i psi)) per pair,
 *   d_dLdc[j] = sum over pairs w (B_j(Kc-Q) - B_j(Kc)),  B_j = d chi / d c_j  (FP64, [8]),
 *   d_dLdtheta[kd] = -sum over Q of w                                  (FP32, [n_K], may be NULL).
 * G is read from the stored double-overlap values (g_mode STORE) or recomputed chunk by chunk
 * from the binned counts (g_mode RECOMPUTE).  normalize must be 0.  The state's counters
 * (STEM_REGION_STATS) keep describing the last sum.  On a state with no FINALIZE since its
 * last ACCUMULATE from frame 0, the adjoint kernels read nothing of it and report the device
 * bit STEM_ESTATE (then d_dLdc and d_dLdtheta are undefined).
 * Errors: STEM_EINVAL, STEM_EWORKSPACE; device bit STEM_ESTATE. */
int ssb_backward(const float* d_dLdphi, const stem_det* det, const stem_scan* scan,
                 const stem_optics* optics, const stem_ssb* ssb, const float* d_theta,
                 void* state, size_t state_bytes, double* d_dLdc, float* d_dLdtheta,
                 int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------------------- */
/* Kernel tracing (measurement support)                                                     */

/* Enable (on != 0, clearing earlier records) or disable per-launch timing: each kernel the
 * library launches is bracketed by two hipEvents recorded on its launch stream. */
int stem_trace_enable(int on);
/* Number of distinct traced kernel names. */
int stem_trace_count(void);
/* Record i: kernel name (NUL-terminated, truncated to name_len), number of launches and the
 * sum of their event-to-event durations in milliseconds.  Waits for the recorded events.
 * STEM_EINVAL for a bad index, STEM_EHIP if an event query fails. */
int stem_trace_get(int i, char* name, size_t name_len, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* STEM4D_H */
