"""Python binding of libstem4d (MI355X / gfx950): event-based 4D-STEM phase contrast.

Argument marshalling only: every computation runs in the HIP kernels of the shared
library; torch provides device memory and the current stream.  The four calls of the
C ABI (include/stem4d.h) keep their names: eer_load_csr, com_dpc, ssb_reconstruct,
ssb_backward.  Importing this package fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

from ._abi import (Det, Dpc, Optics, Scan, Ssb, StemError, lib, LIB_PATH, STEM_FFT_FP32,
                   STEM_DFT_BF16_SPLIT, STEM_DFT_FP16_SPLIT, STEM_G_RECOMPUTE, STEM_G_STORE,
                   STEM_SSB_ACCUMULATE, STEM_SSB_FINALIZE, STEM_SSB_REFOCUS, STEM_SSB_ONESHOT,
                   STEM_REGION_D, STEM_REGION_X, STEM_REGION_T, STEM_REGION_KC, STEM_REGION_STATS, STEM_REGION_PG,
                   STEM_REGION_POFF, STEM_REGION_NPAIR, STEM_ERANGE, STEM_EOFFSETS, STEM_EOVERFLOW,
                   STEM_EWORKSPACE, STEM_EHIP, STEM_ESTATE, STATUS_BITS, strerror, trace_enable,
                   trace_records)

__all__ = [
    "Det", "Scan", "Optics", "Dpc", "Ssb", "StemError", "lib", "LIB_PATH",
    "eer_load_csr", "com_dpc", "com_dpc_workspace_bytes", "ssb_reconstruct", "ssb_backward",
    "ssb_num_pixels", "ssb_state_bytes", "status_tensor", "check_status", "strerror",
    "STEM_FFT_FP32", "STEM_DFT_BF16_SPLIT", "STEM_DFT_FP16_SPLIT", "STEM_G_RECOMPUTE",
    "STEM_G_STORE", "STEM_SSB_ACCUMULATE", "STEM_SSB_FINALIZE", "STEM_SSB_REFOCUS",
    "STEM_SSB_ONESHOT", "SsbState", "SSBPhase", "ssb_state_region", "STEM_REGION_D", "STEM_REGION_X",
    "STEM_REGION_T", "STEM_REGION_KC", "STEM_REGION_STATS", "STEM_REGION_PG", "STEM_REGION_POFF", "STEM_REGION_NPAIR",
    "com_dpc_noalloc", "trace_enable", "trace_records", "STEM_ERANGE", "STEM_EOFFSETS", "STEM_EOVERFLOW",
    "STEM_EWORKSPACE", "STEM_EHIP", "STEM_ESTATE",
    "virtual_annular", "sum_frames", "eer_decode_rle", "ssb_g_panel", "ssb_reconstruct_com",
]


def _p(t):
    """Device/host pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(rc: int, what: str):
    if rc != 0:
        raise StemError(rc, what)


def _dev(t, dtype, name, numel=None):
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")


def status_tensor(device="cuda") -> torch.Tensor:
    """A zeroed int32 device word for the device-side status bits."""
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_status(status: torch.Tensor, what: str = "device status"):
    """Synchronises on the status word and raises if any error bit is set."""
    v = int(status.item())
    if v:
        raise StemError(v, what)


# ----------------------------------------------------------------------------------------------
# a1


def eer_load_csr(h_idx, h_off, frame0: int, n_frames: int, n_events: int, det: Det, d_idx, d_off,
                 d_status=None, stream=None):
    """Copy (h_idx, h_off given, CPU tensors, ideally pinned) or only validate (both None) a
    chunk of frames into the device CSR arrays d_idx (int32) / d_off (int64)."""
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    if (h_idx is None) != (h_off is None):
        raise ValueError("h_idx and h_off must both be given or both be None")
    if h_idx is not None:
        if h_idx.is_cuda or h_off.is_cuda or h_idx.dtype != torch.int32 or h_off.dtype != torch.int64:
            raise ValueError("h_idx/h_off must be int32/int64 host tensors")
        if not (h_idx.is_contiguous() and h_off.is_contiguous()):
            raise ValueError("host tensors must be contiguous")
    rc = lib().eer_load_csr(_p(h_idx), _p(h_off), frame0, n_frames, n_events, ctypes.byref(det),
                            _p(d_idx), _p(d_off), _p(d_status), _stream(stream))
    _check(rc, "eer_load_csr")


def eer_decode_rle(d_dist, d_off, frame0: int, n_frames: int, det: Det, d_idx, d_status=None, stream=None):
    """Run-length form (per-frame distances between ascending hits) -> linear indices d_idx."""
    _dev(d_dist, torch.int32, "d_dist")
    _dev(d_off, torch.int64, "d_off")
    _dev(d_idx, torch.int32, "d_idx")
    rc = lib().eer_decode_rle(_p(d_dist), _p(d_off), frame0, n_frames, ctypes.byref(det), _p(d_idx), _p(d_status),
                              _stream(stream))
    _check(rc, "eer_decode_rle")


# ----------------------------------------------------------------------------------------------
# virtual detectors (Table 1: radial sum, sum of all frames)


def virtual_annular(d_idx, d_off, frame0: int, n_frames: int, det: Det, scan: Scan, r_in, r_out, out,
                    d_status=None, stream=None):
    """Per-frame event counts in annuli r_in[j] <= |k - c| < r_out[j] (pixels): out int32 [n_det*F]."""
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    _dev(out, torch.int32, "out")
    n = len(r_in)
    if len(r_out) != n:
        raise ValueError("r_in and r_out must have the same length")
    F = scan.ny * scan.nx
    if out.numel() < n * F:
        raise ValueError(f"out needs {n * F} elements")
    a = (ctypes.c_double * n)(*[float(v) for v in r_in])
    b = (ctypes.c_double * n)(*[float(v) for v in r_out])
    rc = lib().virtual_annular(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), ctypes.byref(scan), n,
                               a, b, _p(out), _p(d_status), _stream(stream))
    _check(rc, "virtual_annular")


def sum_frames(d_idx, d_off, frame0: int, n_frames: int, det: Det, out_sum, out_mean=None, d_status=None,
               stream=None):
    """Adds the events of frames [frame0, frame0 + n_frames) into out_sum (int32 storage of
    uint32 [H*W]); out_mean (float32 [H*W]), if given, receives the sum / n_frames."""
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    _dev(out_sum, torch.int32, "out_sum")
    if out_sum.numel() < det.W * det.H:
        raise ValueError("out_sum needs W*H elements")
    if out_mean is not None:
        _dev(out_mean, torch.float32, "out_mean")
    rc = lib().sum_frames(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), _p(out_sum), _p(out_mean),
                          _p(d_status), _stream(stream))
    _check(rc, "sum_frames")


# ----------------------------------------------------------------------------------------------
# a2 + a3


def com_dpc_workspace_bytes(scan: Scan) -> int:
    return int(lib().com_dpc_workspace_bytes(ctypes.byref(scan)))


def com_dpc(d_idx, d_off, frame0: int, n_frames: int, det: Det, scan: Scan, optics: Optics | None = None,
            dpc: Dpc | None = None, com64=None, com32=None, counts=None, phase=None, ws=None,
            d_status=None, stream=None):
    """Centre of mass of a frame range; with `phase` given, then the DPC integration."""
    F = scan.ny * scan.nx
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    _dev(com64, torch.float64, "com64", 2 * F)
    _dev(com32, torch.float32, "com32", 2 * F)
    _dev(counts, torch.int32, "counts", F)
    _dev(phase, torch.float32, "phase", F)
    ws_bytes = 0
    if ws is not None:
        _dev(ws, torch.uint8, "ws")
        ws_bytes = ws.numel()
    rc = lib().com_dpc(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), ctypes.byref(scan),
                       ctypes.byref(optics) if optics is not None else None,
                       ctypes.byref(dpc) if dpc is not None else None, _p(com64), _p(com32), _p(counts),
                       _p(phase), _p(ws), ws_bytes, _p(d_status), _stream(stream))
    _check(rc, "com_dpc")


def com_dpc_noalloc(d_idx, d_off, frame0: int, n_frames: int, det: Det, scan: Scan, optics: Optics | None = None,
                    dpc: Dpc | None = None, com64=None, com32=None, counts=None, phase=None, d_status=None,
                    stream=None):
    """com_dpc without a caller workspace (the library's per-device array; calls on one GPU must
    not overlap)."""
    F = scan.ny * scan.nx
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    _dev(com64, torch.float64, "com64", 2 * F)
    _dev(com32, torch.float32, "com32", 2 * F)
    _dev(counts, torch.int32, "counts", F)
    _dev(phase, torch.float32, "phase", F)
    rc = lib().com_dpc_noalloc(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), ctypes.byref(scan),
                               ctypes.byref(optics) if optics is not None else None,
                               ctypes.byref(dpc) if dpc is not None else None, _p(com64), _p(com32), _p(counts),
                               _p(phase), _p(d_status), _stream(stream))
    _check(rc, "com_dpc_noalloc")


# ----------------------------------------------------------------------------------------------
# a4 - a8


def ssb_num_pixels(det: Det, optics: Optics) -> int:
    n = int(lib().ssb_num_pixels(ctypes.byref(det), ctypes.byref(optics)))
    if n < 0:
        raise StemError(-n, "ssb_num_pixels")
    return n


def ssb_state_bytes(det: Det, scan: Scan, optics: Optics, ssb: Ssb) -> int:
    return int(lib().ssb_state_bytes(ctypes.byref(det), ctypes.byref(scan), ctypes.byref(optics),
                                     ctypes.byref(ssb)))


def ssb_state_region(det: Det, scan: Scan, optics: Optics, ssb: Ssb, region: int):
    """(byte offset, byte size) of a region of the sideband state buffer."""
    off, nb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    rc = lib().ssb_state_region(ctypes.byref(det), ctypes.byref(scan), ctypes.byref(optics), ctypes.byref(ssb),
                                region, ctypes.byref(off), ctypes.byref(nb))
    _check(rc, "ssb_state_region")
    return int(off.value), int(nb.value)


def ssb_reconstruct(d_idx, d_off, frame0: int, n_frames: int, det: Det, scan: Scan, optics: Optics,
                    ssb: Ssb, mode: int, state, theta=None, phase=None, T=None, d_status=None,
                    stream=None):
    """Sideband reconstruction step `mode` on a caller-owned state buffer (uint8 CUDA tensor)."""
    F = scan.ny * scan.nx
    if d_idx is not None:
        _dev(d_idx, torch.int32, "d_idx")
        _dev(d_off, torch.int64, "d_off")
    _dev(state, torch.uint8, "state")
    _dev(theta, torch.float32, "theta")
    _dev(phase, torch.float32, "phase", F)
    _dev(T, torch.complex64, "T", F)
    rc = lib().ssb_reconstruct(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), ctypes.byref(scan),
                               ctypes.byref(optics), ctypes.byref(ssb), mode, _p(theta), _p(state),
                               state.numel(), _p(phase), _p(T), _p(d_status), _stream(stream))
    _check(rc, "ssb_reconstruct")


def ssb_reconstruct_com(d_idx, d_off, frame0: int, n_frames: int, det: Det, scan: Scan, optics: Optics,
                        ssb: Ssb, mode: int, state, com64=None, com32=None, counts=None, theta=None, phase=None,
                        T=None, d_status=None, stream=None):
    """ACCUMULATE or ONESHOT that also writes the frames' centre of mass (as com_dpc) from the
    same pass over the events."""
    F = scan.ny * scan.nx
    _dev(d_idx, torch.int32, "d_idx")
    _dev(d_off, torch.int64, "d_off")
    _dev(state, torch.uint8, "state")
    _dev(theta, torch.float32, "theta")
    _dev(phase, torch.float32, "phase", F)
    _dev(T, torch.complex64, "T", F)
    _dev(com64, torch.float64, "com64", 2 * F)
    _dev(com32, torch.float32, "com32", 2 * F)
    _dev(counts, torch.int32, "counts", F)
    rc = lib().ssb_reconstruct_com(_p(d_idx), _p(d_off), frame0, n_frames, ctypes.byref(det), ctypes.byref(scan),
                                   ctypes.byref(optics), ctypes.byref(ssb), mode, _p(theta), _p(state),
                                   state.numel(), _p(phase), _p(T), _p(com64), _p(com32), _p(counts),
                                   _p(d_status), _stream(stream))
    _check(rc, "ssb_reconstruct_com")


def ssb_backward(dLdphi, det: Det, scan: Scan, optics: Optics, ssb: Ssb, state, dLdc, theta=None,
                 dLdtheta=None, d_status=None, stream=None):
    """Adjoint of the sideband phase: fills dLdc (float64 [8]) and dLdtheta (float32 [n_K])."""
    F = scan.ny * scan.nx
    _dev(dLdphi, torch.float32, "dLdphi", F)
    _dev(state, torch.uint8, "state")
    _dev(dLdc, torch.float64, "dLdc", 8)
    _dev(theta, torch.float32, "theta")
    _dev(dLdtheta, torch.float32, "dLdtheta")
    rc = lib().ssb_backward(_p(dLdphi), ctypes.byref(det), ctypes.byref(scan), ctypes.byref(optics),
                            ctypes.byref(ssb), _p(theta), _p(state), state.numel(), _p(dLdc), _p(dLdtheta),
                            _p(d_status), _stream(stream))
    _check(rc, "ssb_backward")


def ssb_g_panel(det: Det, scan: Scan, optics: Optics, ssb: Ssb, state, qs, out, stream=None):
    """G(K, Q) of the kept bins at the scan frequencies qs = [(my, mx), ...] as binned detector
    images: out complex64 [len(qs), H/bin, W/bin], 0 on dropped bins."""
    _dev(state, torch.uint8, "state")
    n = len(qs)
    nby, nbx = det.H // det.bin, det.W // det.bin
    _dev(out, torch.complex64, "out", n * nby * nbx)
    my = (ctypes.c_int32 * max(n, 1))(*[int(q[0]) for q in qs])
    mx = (ctypes.c_int32 * max(n, 1))(*[int(q[1]) for q in qs])
    rc = lib().ssb_g_panel(ctypes.byref(det), ctypes.byref(scan), ctypes.byref(optics), ctypes.byref(ssb),
                           _p(state), state.numel(), n, my, mx, _p(out), _stream(stream))
    _check(rc, "ssb_g_panel")


# ----------------------------------------------------------------------------------------------
# stateful convenience + autograd


class SsbState:
    """Owns a sideband state buffer for one geometry and runs the reconstruction on it."""

    def __init__(self, det: Det, scan: Scan, optics: Optics, ssb: Ssb | None = None, device="cuda"):
        self.det, self.scan, self.optics = det, scan, optics
        self.ssb = ssb if ssb is not None else Ssb(STEM_FFT_FP32, 0, STEM_G_STORE, 8)
        self.n_k = ssb_num_pixels(det, optics)
        nbytes = ssb_state_bytes(det, scan, optics, self.ssb)
        if nbytes == 0:
            raise StemError(1, "ssb_state_bytes: invalid geometry")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.status = status_tensor(device)
        self.F = scan.ny * scan.nx

    def region(self, which: int) -> torch.Tensor:
        """A uint8 view of one region of the state buffer (see ssb_state_region)."""
        off, nb = ssb_state_region(self.det, self.scan, self.optics, self.ssb, which)
        return self.state[off:off + nb]

    def pair_count(self) -> int:
        """Double-overlap (pixel, Q) pairs of the last sum (waits for the stream)."""
        return int(self.region(STEM_REGION_STATS).view(torch.int64)[0].item())

    def stats(self) -> list:
        """The four uint64 counters of the state (pairs, partial sums of T, reserved)."""
        return [int(v) for v in self.region(STEM_REGION_STATS).view(torch.int64).cpu().tolist()]

    def optics_with(self, c) -> Optics:
        o = Optics.from_values(self.optics.lam, self.optics.r_bf, self.optics.dk, c)
        return o

    def accumulate(self, d_idx, d_off, frame0: int, n_frames: int, com64=None, com32=None, counts=None,
                   stream=None):
        """Bin and row-transform whole scan rows; with a centre-of-mass output, the same pass over
        the events also writes the frames' centre of mass (as com_dpc)."""
        if com64 is None and com32 is None and counts is None:
            ssb_reconstruct(d_idx, d_off, frame0, n_frames, self.det, self.scan, self.optics, self.ssb,
                            STEM_SSB_ACCUMULATE, self.state, d_status=self.status, stream=stream)
        else:
            ssb_reconstruct_com(d_idx, d_off, frame0, n_frames, self.det, self.scan, self.optics, self.ssb,
                                STEM_SSB_ACCUMULATE, self.state, com64=com64, com32=com32, counts=counts,
                                d_status=self.status, stream=stream)

    def finalize(self, c=None, theta=None, phase=None, T=None, stream=None):
        o = self.optics if c is None else self.optics_with(c)
        ssb_reconstruct(None, None, 0, 0, self.det, self.scan, o, self.ssb, STEM_SSB_FINALIZE, self.state,
                        theta=theta, phase=phase, T=T, d_status=self.status, stream=stream)

    def refocus(self, c=None, theta=None, phase=None, T=None, stream=None):
        o = self.optics if c is None else self.optics_with(c)
        ssb_reconstruct(None, None, 0, 0, self.det, self.scan, o, self.ssb, STEM_SSB_REFOCUS, self.state,
                        theta=theta, phase=phase, T=T, d_status=self.status, stream=stream)

    def oneshot(self, d_idx, d_off, c=None, theta=None, phase=None, T=None, com64=None, com32=None, counts=None,
                stream=None):
        o = self.optics if c is None else self.optics_with(c)
        if com64 is None and com32 is None and counts is None:
            ssb_reconstruct(d_idx, d_off, 0, self.F, self.det, self.scan, o, self.ssb, STEM_SSB_ONESHOT,
                            self.state, theta=theta, phase=phase, T=T, d_status=self.status, stream=stream)
        else:
            ssb_reconstruct_com(d_idx, d_off, 0, self.F, self.det, self.scan, o, self.ssb, STEM_SSB_ONESHOT,
                                self.state, com64=com64, com32=com32, counts=counts, theta=theta, phase=phase,
                                T=T, d_status=self.status, stream=stream)

    def g_panel(self, qs, stream=None) -> torch.Tensor:
        """G at the scan frequencies qs = [(my, mx), ...] as binned detector images
        (complex64 [len(qs), H/bin, W/bin]); call after finalize, oneshot or refocus."""
        out = torch.empty(len(qs), self.det.H // self.det.bin, self.det.W // self.det.bin, dtype=torch.complex64,
                          device=self.state.device)
        ssb_g_panel(self.det, self.scan, self.optics, self.ssb, self.state, qs, out, stream=stream)
        return out

    def backward(self, dLdphi, c=None, theta=None, with_theta=True, stream=None):
        o = self.optics if c is None else self.optics_with(c)
        dc = torch.empty(8, dtype=torch.float64, device=self.state.device)
        dth = torch.empty(self.n_k, dtype=torch.float32, device=self.state.device) if with_theta else None
        ssb_backward(dLdphi, self.det, self.scan, o, self.ssb, self.state, dc, theta=theta, dLdtheta=dth,
                     d_status=self.status, stream=stream)
        return dc, dth


class SSBPhase(torch.autograd.Function):
    """phi = SSB phase for aberration coefficients c (float64 [8]) and probe phase theta
    (float32 [n_K]) on the accumulated events of `st` (an SsbState in G-store or
    G-recompute mode).  backward returns dL/dc and dL/dtheta from the hand-written adjoint."""

    @staticmethod
    def forward(ctx, c, theta, st: SsbState):
        cv = [float(v) for v in c.detach().cpu().tolist()]
        th = theta.detach().contiguous() if theta is not None else None
        phase = torch.empty(st.scan.ny, st.scan.nx, dtype=torch.float32, device=st.state.device)
        st.refocus(cv, th, phase=phase) if getattr(st, "_finalized", False) else st.finalize(cv, th, phase=phase)
        st._finalized = st.ssb.g_mode == STEM_G_STORE
        ctx.st, ctx.cv, ctx.th = st, cv, th
        ctx.c_dtype, ctx.c_device = c.dtype, c.device
        return phase

    @staticmethod
    def backward(ctx, gphi):
        st = ctx.st
        dc, dth = st.backward(gphi.detach().contiguous().to(torch.float32), ctx.cv, ctx.th,
                              with_theta=ctx.th is not None)
        return dc.to(ctx.c_device, ctx.c_dtype), dth, None
