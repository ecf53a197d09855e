"""Shared helpers for the GPU parity tests: parameter structs, data movement, oracle runs."""
from __future__ import annotations

import math

import numpy as np
import torch

import paper_2104_06336_amd as stem
from oracle import dpc as odpc
from oracle import eer as oeer
from oracle import ssb as ossb


def structs(wl, c=None, bin_=None):
    H, W = wl.det
    det = stem.Det(W, H, W // 2, H // 2, wl.bin if bin_ is None else bin_)
    scan = stem.Scan(wl.scan[0], wl.scan[1], wl.step)
    optics = stem.Optics.from_values(wl.lam, wl.r_bf, wl.dk, c if c is not None else (0.0,) * 8)
    return det, scan, optics


def to_device(idx, off, device="cuda"):
    """CSR arrays (numpy or torch) -> contiguous device tensors."""
    i = torch.as_tensor(np.asarray(idx) if not torch.is_tensor(idx) else idx).to(device, torch.int32).contiguous()
    o = torch.as_tensor(np.asarray(off) if not torch.is_tensor(off) else off).to(device, torch.int64).contiguous()
    return i, o


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    den = np.sqrt(np.sum(np.abs(b) ** 2))
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2)) / (den if den > 0 else 1.0))


def gpu_com(d_idx, d_off, wl, frame0=0, n_frames=None, phase=False, dpc_params=None):
    det, scan, optics = structs(wl)
    F = wl.n_frames
    n_frames = F - frame0 if n_frames is None else n_frames
    dev = d_idx.device
    com64 = torch.zeros(2 * F, dtype=torch.float64, device=dev)
    com32 = torch.zeros(2 * F, dtype=torch.float32, device=dev)
    counts = torch.zeros(F, dtype=torch.int32, device=dev)
    status = stem.status_tensor(dev)
    out = {}
    ph = ws = None
    dp = dpc_params or stem.Dpc(0.5, 0.0, 0.0, 10)
    if phase:
        ph = torch.zeros(F, dtype=torch.float32, device=dev)
        ws = torch.empty(stem.com_dpc_workspace_bytes(scan), dtype=torch.uint8, device=dev)
    stem.com_dpc(d_idx, d_off, frame0, n_frames, det, scan, optics, dp, com64=com64, com32=com32, counts=counts,
                 phase=ph, ws=ws, d_status=status)
    torch.cuda.synchronize()
    out["status"] = int(status.item())
    out["com64"] = com64.cpu().numpy().reshape(2, F)
    out["com32"] = com32.cpu().numpy().reshape(2, F)
    out["counts"] = counts.cpu().numpy()
    if phase:
        out["phase"] = ph.cpu().numpy().reshape(wl.scan)
    return out


def oracle_dpc(idx, off, wl, mu=0.5, lam1=0.0, lam2=0.0, n_iter=10):
    H, W = wl.det
    cx, cy, *_ = oeer.com(idx, off, W, H)
    ny, nx = wl.scan
    return odpc.com_dpc(cx.reshape(ny, nx), cy.reshape(ny, nx), wl.dk, wl.step, mu=mu, lam1=lam1,
                        lam2=lam2, n_iter=n_iter)


def oracle_ssb(idx, off, wl, c=(0.0,) * 8, theta=None, normalize=False, direct=False):
    """Oracle D, Kc, G, T, phi for one acquisition."""
    H, W = wl.det
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    D = oeer.bin_counts(idx, off, W, wl.bin, lut)
    ny, nx = wl.scan
    phi, T, G = ossb.ssb_forward(D, kc, ny, nx, wl.step, wl.dk, wl.lam, wl.r_bf, c, theta, normalize, direct)
    return {"D": D, "kc": kc, "G": G, "T": T, "phi": phi}


def gpu_ssb(d_idx, d_off, wl, c=(0.0,) * 8, theta=None, normalize=0, g_mode=stem.STEM_G_STORE, d_bits=8,
            chunk_rows=None, precision=stem.STEM_FFT_FP32, scratch_mib=0):
    det, scan, optics = structs(wl, c)
    ssb = stem.Ssb(precision, normalize, g_mode, d_bits, scratch_mib)
    st = stem.SsbState(det, scan, optics, ssb, device=d_idx.device)
    F = wl.n_frames
    ny, nx = wl.scan
    phase = torch.zeros(F, dtype=torch.float32, device=d_idx.device)
    T = torch.zeros(F, dtype=torch.complex64, device=d_idx.device)
    th = None if theta is None else torch.as_tensor(theta, dtype=torch.float32, device=d_idx.device)
    if chunk_rows is None:
        st.oneshot(d_idx, d_off, c=c, theta=th, phase=phase, T=T)
    else:
        for r0 in range(0, ny, chunk_rows):
            nr = min(chunk_rows, ny - r0)
            st.accumulate(d_idx, d_off, r0 * nx, nr * nx)
        st.finalize(c=c, theta=th, phase=phase, T=T)
    torch.cuda.synchronize()
    return st, {"status": int(st.status.item()), "phi": phase.cpu().numpy().reshape(ny, nx),
                "T": T.cpu().numpy().reshape(ny, nx)}


def state_D(st, wl):
    raw = st.region(stem.STEM_REGION_D)
    dt = torch.uint8 if st.ssb.d_bits == 8 else torch.int16
    D = raw.view(dt).cpu().numpy()
    if st.ssb.d_bits == 16:
        D = D.view(np.uint16)
    return D.reshape(st.n_k, wl.n_frames).astype(np.int64)


def state_X(st, wl):
    """Row-transformed cube X[kd][mx][ry] (STEM_G_STORE, after ACCUMULATE) -> array [kd][ry][mx_half]."""
    ny, nx = wl.scan
    raw = st.region(stem.STEM_REGION_X).view(torch.complex64).cpu().numpy()
    return raw.reshape(st.n_k, nx // 2 + 1, ny).transpose(0, 2, 1)


def oracle_row_dft(D, wl):
    """The DFT along rx of every row of the oracle's cube, first Nx/2 + 1 frequencies: [kd][ry][mx]."""
    ny, nx = wl.scan
    D3 = ossb.cube(D, ny, nx).astype(np.complex128)
    return np.matmul(D3, ossb.dft_matrix(nx).T[None])[:, :, :nx // 2 + 1]


def state_pruned(st):
    """(pruned G values, offsets) of a STEM_G_STORE state after FINALIZE."""
    poff = st.region(stem.STEM_REGION_POFF).view(torch.int64).cpu().numpy()
    n = int(poff[-1])
    pg = st.region(stem.STEM_REGION_PG).view(torch.complex64)[:n].cpu().numpy()
    return pg, poff


def oracle_pruned(G, kc, wl):
    """G on the double-overlap pairs in the pruned layout, from the oracle's full G[kd][my][mx] and
    set (ossb.double_overlap): column mx in [0, Nx) major, then pixel, then ascending signed my;
    and the offsets of every (column, pixel) run."""
    ny, nx = wl.scan
    qx, qy = ossb.scan_q_grid(ny, nx, wl.step, wl.dk)
    order = np.argsort(ossb.signed_freq_index(ny), kind="stable")  # rows by ascending signed my
    masks, gs = [], []
    r2 = float(wl.r_bf) * float(wl.r_bf)
    for kd in range(len(kc)):
        masks.append(ossb.double_overlap(float(kc[kd, 0]), float(kc[kd, 1]), qx, qy, r2)[order].T)  # [mx][iy]
        gs.append(G[kd][order].T)
    vals, sizes = [], []
    for mx in range(nx):
        for kd in range(len(kc)):
            vals.append(gs[kd][mx][masks[kd][mx]])
            sizes.append(int(masks[kd][mx].sum()))
    poff = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))])
    return np.concatenate(vals), poff


def state_npair(st, wl):
    """Per-Q pair counts (after a FINALIZE with normalize = 1) as [my][mx]."""
    ny, nx = wl.scan
    return st.region(stem.STEM_REGION_NPAIR).view(torch.int32).cpu().numpy().reshape(nx, ny).T


def state_kc(st):
    return st.region(stem.STEM_REGION_KC).view(torch.float64).cpu().numpy().reshape(st.n_k, 2)


def q_error_scale(G_ref, kc, wl):
    """Per-Q scale of the error of T: the root sum of squares of its summands |G(K, Q)| over the
    double-overlap set, plus sqrt(n(Q)) times the rms of G (the floor of a transform's rounding for
    small elements).  A wrong membership or a wrong term at a single Q moves the error relative to
    this scale by about 1/sqrt(n(Q))."""
    s2, npair = ossb.ssb_sum(np.abs(G_ref) ** 2, kc, wl.step, wl.dk, wl.lam, wl.r_bf)
    g_rms = float(np.sqrt(np.mean(np.abs(G_ref) ** 2)))
    return np.sqrt(np.abs(s2)) + np.sqrt(npair) * g_rms + 1e-30


def per_q_error(T, T_ref, scale):
    """Largest error of T over the scan frequencies, each relative to its own scale."""
    return float(np.max(np.abs(np.asarray(T) - T_ref) / scale))
