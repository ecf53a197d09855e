"""Oracle: per-frame reductions on linear-index electron events (FP64 / exact integers).

Test infrastructure only (see the package docstring).  Each function restates a
definition of the paper in plain numpy; nothing here is shared with the HIP path.

Event encoding (Fig. 1b, Sec. II): a frame is the list of linear indices
k = ky*W + kx of its electron hits; a dataset is a CSR pair (idx[C], off[F+1]),
frame f holding idx[off[f]:off[f+1]].  Frames follow raster scan order.
"""
from __future__ import annotations

import numpy as np


def frame_counts(off: np.ndarray) -> np.ndarray:
    """N_f = off[f+1] - off[f]: the number of electrons recorded in frame f (Table 1, Sec. III)."""
    off = np.asarray(off, dtype=np.int64)
    return off[1:] - off[:-1]


def frame_of_event(off: np.ndarray) -> np.ndarray:
    """Frame number of every event (the CSR row index)."""
    n = frame_counts(off)
    return np.repeat(np.arange(n.size, dtype=np.int64), n)


def dense_frames(idx: np.ndarray, off: np.ndarray, W: int, H: int) -> np.ndarray:
    """The dense 4D cube rho[f, ky, kx] = #events of frame f on pixel (kx, ky).

    This is the 'dense format' column of Table 1; it exists here only to check the
    event-based reductions by brute force on tiny inputs.
    """
    F = len(off) - 1
    rho = np.zeros((F, H, W), dtype=np.int64)
    for f in range(F):
        for k in np.asarray(idx[off[f]:off[f + 1]], dtype=np.int64):
            rho[f, k // W, k % W] += 1
    return rho


def com(idx: np.ndarray, off: np.ndarray, W: int, H: int, cx: int | None = None,
        cy: int | None = None):
    """Centre of mass of each frame from its events (Eq. 4, Table 1 'center of mass').

    Eq. 4 integrates the intensity times the momentum coordinate; dividing by the
    frame's electron count gives the centre of mass.  Coordinates are detector
    pixels relative to the zero-frequency pixel (cx, cy) = (W/2, H/2) by default.

    The first moments Sx = sum(kx - cx), Sy = sum(ky - cy) are exact int64 sums;
    each component is then one IEEE float64 division Sx / N_f.  A frame with no
    events has centre of mass 0.

    Returns (com_x[F], com_y[F], Sx[F], Sy[F], N[F]).
    """
    cx = W // 2 if cx is None else cx
    cy = H // 2 if cy is None else cy
    k = np.asarray(idx, dtype=np.int64)
    dx = k % W - cx
    dy = k // W - cy
    # exclusive prefix sums: the sum over a frame is a difference of two prefix values
    px = np.concatenate([[0], np.cumsum(dx)])
    py = np.concatenate([[0], np.cumsum(dy)])
    off = np.asarray(off, dtype=np.int64)
    sx = px[off[1:]] - px[off[:-1]]
    sy = py[off[1:]] - py[off[:-1]]
    n = frame_counts(off)
    with np.errstate(invalid="ignore", divide="ignore"):
        com_x = np.where(n > 0, sx.astype(np.float64) / np.maximum(n, 1).astype(np.float64), 0.0)
        com_y = np.where(n > 0, sy.astype(np.float64) / np.maximum(n, 1).astype(np.float64), 0.0)
    return com_x, com_y, sx, sy, n


def com_dense(rho: np.ndarray, cx: int, cy: int):
    """Brute-force centre of mass of dense frames rho[f, ky, kx] (Eq. 4 over all pixels)."""
    F, H, W = rho.shape
    xs = np.arange(W, dtype=np.int64) - cx
    ys = np.arange(H, dtype=np.int64) - cy
    n = rho.sum(axis=(1, 2))
    sx = (rho * xs[None, None, :]).sum(axis=(1, 2))
    sy = (rho * ys[None, :, None]).sum(axis=(1, 2))
    com_x = np.array([sx[f] / n[f] if n[f] else 0.0 for f in range(F)])
    com_y = np.array([sy[f] / n[f] if n[f] else 0.0 for f in range(F)])
    return com_x, com_y, sx, sy, n


def bin_geometry(W: int, H: int, b: int, r_bf: float, cx: int | None = None, cy: int | None = None):
    """Binned pixels kept for the sideband path (Sec. IV: centre, crop and bin from EER).

    Bin (bx, by) collects unbinned pixels kx in [b*bx, b*bx + b), ky in [b*by, b*by + b);
    its centre relative to the zero-frequency pixel is
    Kc = (b*bx + (b-1)/2 - cx, b*by + (b-1)/2 - cy) unbinned pixels.  A bin is kept
    (the crop) iff its centre lies strictly inside the bright-field disk,
    Kc.Kc < r_bf^2; the values are multiples of 1/2, so the test is exact.  Kept bins
    are numbered kd = 0, 1, ... in raster (by, bx) order.

    Returns (Kc[n_K, 2] as (x, y) float64, lut[H/b, W/b] int64 with -1 for dropped bins).
    """
    if W % b or H % b:
        raise ValueError("detector size must be a multiple of the binning factor")
    cx = W // 2 if cx is None else cx
    cy = H // 2 if cy is None else cy
    nbx, nby = W // b, H // b
    lut = -np.ones((nby, nbx), dtype=np.int64)
    kc = []
    r2 = float(r_bf) * float(r_bf)
    for by in range(nby):
        for bx in range(nbx):
            kcx = b * bx + (b - 1) / 2.0 - cx
            kcy = b * by + (b - 1) / 2.0 - cy
            if kcx * kcx + kcy * kcy < r2:
                lut[by, bx] = len(kc)
                kc.append((kcx, kcy))
    return np.array(kc, dtype=np.float64).reshape(-1, 2), lut


def bin_counts(idx: np.ndarray, off: np.ndarray, W: int, b: int, lut: np.ndarray) -> np.ndarray:
    """Binned, cropped count cube D[kd, f] = #events of frame f in kept bin kd (Table 1 'bin', 'crop').

    Each event costs O(1): kx = k mod W, ky = k div W, (bx, by) = (kx div b, ky div b),
    kd = lut[by, bx]; events in dropped bins are discarded.
    """
    k = np.asarray(idx, dtype=np.int64)
    F = len(off) - 1
    kd = lut[(k // W) // b, (k % W) // b]
    f = frame_of_event(off)
    keep = kd >= 0
    D = np.zeros((int(lut.max()) + 1, F), dtype=np.int64)
    np.add.at(D, (kd[keep], f[keep]), 1)
    return D


def bin_dense(rho: np.ndarray, b: int, lut: np.ndarray) -> np.ndarray:
    """Brute-force binning of dense frames: sum b x b pixel blocks, keep lut >= 0."""
    F, H, W = rho.shape
    blocks = rho.reshape(F, H // b, b, W // b, b).sum(axis=(2, 4))
    n_k = int(lut.max()) + 1
    D = np.zeros((n_k, F), dtype=np.int64)
    for by in range(H // b):
        for bx in range(W // b):
            if lut[by, bx] >= 0:
                D[lut[by, bx]] = blocks[:, by, bx]
    return D


def radial_sum(idx: np.ndarray, off: np.ndarray, W: int, H: int, r_in, r_out, cx: int | None = None,
               cy: int | None = None) -> np.ndarray:
    """Virtual annular detectors from events (Table 1 'radial sum', Sec. III).

    For each annulus j and frame f: the number of events of f whose pixel lies at squared
    distance d2 = (kx - cx)^2 + (ky - cy)^2 from the zero-frequency pixel with
    r_in[j]^2 <= d2 < r_out[j]^2 (d2 is an exact integer, the radii squared in float64).
    Cost O(C) from events, against O((r_out^2 - r_in^2) F) from dense frames.

    Returns int64 [n_det, F].
    """
    cx = W // 2 if cx is None else cx
    cy = H // 2 if cy is None else cy
    k = np.asarray(idx, dtype=np.int64)
    d2 = (k % W - cx) ** 2 + (k // W - cy) ** 2
    f = frame_of_event(off)
    F = len(off) - 1
    out = np.zeros((len(r_in), F), dtype=np.int64)
    for j, (a, b) in enumerate(zip(r_in, r_out)):
        a2, b2 = float(a) * float(a), float(b) * float(b)
        inside = (d2 >= a2) & (d2 < b2)
        out[j] = np.bincount(f[inside], minlength=F)
    return out


def sum_frames(idx: np.ndarray, off: np.ndarray, W: int, H: int, frame0: int = 0,
               n_frames: int | None = None) -> np.ndarray:
    """Sum of the frames [frame0, frame0 + n_frames) (Table 1 'sum all frames'): the
    position-averaged diffraction pattern (PACBED) up to the factor 1/n_frames, or, over frames
    in vacuum, the average probe.  Each event adds one count to its pixel.

    Returns int64 [H, W].
    """
    F = len(off) - 1
    n_frames = F - frame0 if n_frames is None else n_frames
    k = np.asarray(idx[off[frame0]:off[frame0 + n_frames]], dtype=np.int64)
    return np.bincount(k, minlength=W * H).reshape(H, W)


def rle_encode(idx: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Run-length form of the events (Fig. 1c): within each frame the indices in ascending order,
    stored as their distances d_0 = k_0, d_i = k_i - k_(i-1) (a repeated pixel gives 0)."""
    k = np.asarray(idx, dtype=np.int64).copy()
    d = np.empty_like(k)
    for f in range(len(off) - 1):
        seg = np.sort(k[off[f]:off[f + 1]])
        if seg.size:
            d[off[f]:off[f + 1]] = np.diff(seg, prepend=0)
    return d


def rle_decode(dist: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Linear indices from the run-length form (Table 1: re-coding costs O(C)): k_i is the sum of
    the frame's distances up to and including i (a prefix sum restarted at every frame)."""
    d = np.asarray(dist, dtype=np.int64)
    k = np.empty_like(d)
    for f in range(len(off) - 1):
        k[off[f]:off[f + 1]] = np.cumsum(d[off[f]:off[f + 1]])
    return k
