"""Seeded synthetic electron-event (EER) data shaped like 4D Camera acquisitions.

Input generator shared by the tests, the oracle checks and the benchmark.  It holds
none of the reconstruction arithmetic (no centre of mass, binning, scan-space
transform, sideband sum or phase integration): it simulates the measurement of
Eq. 1 (projection approximation: a frame is |FFT_r[a(r - R) T(r)]|^2) and draws
electron events from it, stored in linear-index encoding (Fig. 1b; Sec. II):
one int32 index k = ky*W + kx per event and int64 per-frame CSR offsets, frames
in raster scan order f = ry*Nx + rx.

Conventions (numpy's): forward FFT carries exp(-2*pi*i k.r); the probe is
a = IFFT(A) with A(k) = aperture(k) * exp(-i chi(k)); the object is
T = exp(i phi).  The detector's zero-frequency pixel is (W/2, H/2).

The forward model runs on a simulation grid of S x S pixels with the detector's
angular sampling dk, centred in the W x H detector.  With S = W this is the full
detector; a smaller S (used for the 576 x 576 workloads, S = 192 > 1.6 k0)
keeps every pixel that the band-limited exit wave reaches while making the
per-frame FFT 9x cheaper.  Event indices always address the full W x H detector.

Everything runs in torch on the requested device (CPU float64, or a GPU in
float32 for the large workloads).  Object atoms come from a numpy RNG seeded by
`obj_seed`, so the object is identical on every device; electron draws use a
torch.Generator seeded by `event_seed`.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from dataclasses import dataclass, field

import numpy as np
import torch

# Relativistic electron wavelength at 300 kV in angstrom (1.97 pm).
LAMBDA_300KV = 0.0196875


@dataclass(frozen=True)
class Workload:
    """Geometry and dose of one synthetic acquisition."""

    name: str
    scan: tuple  # (Ny, Nx) probe positions
    step: float  # scan step in angstrom
    det: tuple  # (H, W) detector pixels
    r_bf: float  # bright-field disk radius in unbinned detector pixels
    mean_e: float  # mean electrons per frame
    bin: int  # detector binning factor used by the sideband path
    sim: int  # simulation grid edge S (centred inside the detector)
    alpha: float = 0.025  # convergence semi-angle, rad
    lam: float = LAMBDA_300KV  # wavelength, angstrom
    aberr: tuple = (0.0,) * 8  # C1, A1a, A1b, B2a, B2b, A2a, A2b, C3 in angstrom
    obj_seed: int = 1234
    event_seed: int = 5678
    atom_density: float = 0.1  # atoms per square angstrom
    atom_sigma: float = 0.5  # angstrom
    peak_phase: float = 0.1  # rad

    @property
    def k0(self) -> float:
        """Bright-field disk radius alpha/lambda in 1/angstrom."""
        return self.alpha / self.lam

    @property
    def dk(self) -> float:
        """Detector pixel size in 1/angstrom."""
        return self.k0 / self.r_bf

    @property
    def dx(self) -> float:
        """Real-space pixel of the simulation grid in angstrom."""
        return 1.0 / (self.sim * self.dk)

    @property
    def n_frames(self) -> int:
        return self.scan[0] * self.scan[1]

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five acquisitions of the evaluation plan (Sec. IV, V; 4D Camera geometry).
C4_TRUE_ABERRATIONS = (50.0, 20.0, 20.0, 300.0, 300.0, 300.0, 300.0, 1.0e4)

WORKLOADS = {
    "small": Workload("small: scan 32x32, detector 64x64, r_bf 16 px, 20 e/frame",
                      (32, 32), 0.2, (64, 64), 16.0, 20.0, 1, 64),
    "scan256": Workload("scan 256x256, detector 576x576 binned 4x, 100 e/frame",
                        (256, 256), 0.2, (576, 576), 60.0, 100.0, 4, 192),
    "scan1024": Workload("scan 1024x1024, detector 576x576 binned 8x, 40 e/frame",
                         (1024, 1024), 0.2, (576, 576), 60.0, 40.0, 8, 192),
    "aberrated512": Workload("scan 512x512, detector 576x576 binned 6x, 60 e/frame, aberrated probe",
                             (512, 512), 0.2, (576, 576), 60.0, 60.0, 6, 192,
                             aberr=C4_TRUE_ABERRATIONS),
}


@dataclass
class EventData:
    """Linear-index EER in CSR form plus the ground truth that produced it."""

    wl: Workload
    idx: torch.Tensor  # int32 [C]
    off: torch.Tensor  # int64 [F+1]
    phase_obj: np.ndarray  # float64 object phase on the simulation grid
    pad: float  # object pixel of the probe centre at R = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_events(self) -> int:
        return int(self.idx.numel())

    def numpy(self):
        return (self.idx.detach().cpu().numpy(), self.off.detach().cpu().numpy())

    def sha256(self) -> str:
        h = hashlib.sha256()
        i, o = self.numpy()
        h.update(np.ascontiguousarray(i).tobytes())
        h.update(np.ascontiguousarray(o).tobytes())
        return h.hexdigest()

    def truth_at_scan(self) -> np.ndarray:
        """Object phase at every probe centre, bilinear, shape (Ny, Nx)."""
        wl = self.wl
        ny, nx = wl.scan
        py = np.arange(ny) * (wl.step / wl.dx) + self.pad
        px = np.arange(nx) * (wl.step / wl.dx) + self.pad
        y0 = np.floor(py).astype(np.int64)
        x0 = np.floor(px).astype(np.int64)
        fy = (py - y0)[:, None]
        fx = (px - x0)[None, :]
        p = self.phase_obj
        return ((1 - fy) * (1 - fx) * p[np.ix_(y0, x0)] + (1 - fy) * fx * p[np.ix_(y0, x0 + 1)]
                + fy * (1 - fx) * p[np.ix_(y0 + 1, x0)] + fy * fx * p[np.ix_(y0 + 1, x0 + 1)])


# ----------------------------------------------------------------------------------------------
# Probe optics (the generator's own copy: it simulates the microscope, Eq. 1)


def _probe_phase(wl: Workload, ky_px: np.ndarray, kx_px: np.ndarray) -> np.ndarray:
    """Aberration phase of the simulated probe, polynomial expansion in omega = lambda*k."""
    c1, a1a, a1b, b2a, b2b, a2a, a2b, c3 = (float(v) for v in wl.aberr)
    wx = wl.lam * (kx_px * wl.dk)
    wy = wl.lam * (ky_px * wl.dk)
    w2 = wx * wx + wy * wy
    poly = (0.5 * c1 * w2 + 0.5 * a1a * (wx * wx - wy * wy) + a1b * wx * wy
            + (b2a * w2 * wx + b2b * w2 * wy) / 3.0
            + (a2a * (wx ** 3 - 3.0 * wx * wy * wy) + a2b * (3.0 * wx * wx * wy - wy ** 3)) / 3.0
            + 0.25 * c3 * w2 * w2)
    return (2.0 * math.pi / wl.lam) * poly


def probe_spectrum(wl: Workload) -> np.ndarray:
    """A(k) on the S x S grid in FFT (unshifted) order: disk(|k| < r_bf) * exp(-i chi)."""
    s = wl.sim
    f = np.fft.fftfreq(s) * s  # integer frequency index
    ky, kx = np.meshgrid(f, f, indexing="ij")
    aperture = (kx * kx + ky * ky) < wl.r_bf ** 2
    return aperture * np.exp(-1j * _probe_phase(wl, ky, kx))


# ----------------------------------------------------------------------------------------------
# Objects


def _object_shape(wl: Workload) -> tuple:
    ny, nx = wl.scan
    pad = wl.sim / 2.0 + 2.0
    ext_y = int(math.ceil((ny - 1) * wl.step / wl.dx + 2 * pad + 2))
    ext_x = int(math.ceil((nx - 1) * wl.step / wl.dx + 2 * pad + 2))
    return (ext_y, ext_x), pad


def atoms_phase(wl: Workload) -> tuple:
    """Gaussian atoms at uniform random positions, rescaled to the requested peak phase."""
    (ey, ex), pad = _object_shape(wl)
    rng = np.random.default_rng(wl.obj_seed)
    area = ey * ex * wl.dx * wl.dx
    n_atoms = max(1, int(round(area * wl.atom_density)))
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 2)) * np.array([ey, ex])
    sig = wl.atom_sigma / wl.dx  # sigma in pixels
    h = int(math.ceil(4.0 * sig))
    # padded canvas: canvas[y + h, x + h] holds object pixel (y, x)
    canvas = np.zeros((ey + 2 * h + 2, ex + 2 * h + 2))
    o = np.arange(-h, h + 2)
    for j in range(n_atoms):
        cy, cx = pos[j]
        iy, ix = int(math.floor(cy)), int(math.floor(cx))
        yy = (iy + o) - cy
        xx = (ix + o) - cx
        patch = np.exp(-(yy[:, None] ** 2 + xx[None, :] ** 2) / (2 * sig * sig))
        canvas[iy:iy + 2 * h + 2, ix:ix + 2 * h + 2] += patch
    phase = canvas[h:h + ey, h:h + ex]
    phase *= wl.peak_phase / phase.max()
    return phase, pad


def ramp_phase(wl: Workload, g_px: tuple) -> tuple:
    """Linear phase 2*pi*(g.r) with g = (gy, gx) detector pixels (T = exp(2 pi i g.r))."""
    (ey, ex), pad = _object_shape(wl)
    gy, gx = (g * wl.dk for g in g_px)
    y = np.arange(ey) * wl.dx
    x = np.arange(ex) * wl.dx
    return 2 * math.pi * (gy * y[:, None] + gx * x[None, :]), pad


def cosine_phase(wl: Workload, amp: float, period_scan_px: tuple) -> tuple:
    """amp * cos(2 pi (y/py + x/px)) with periods given in scan steps."""
    (ey, ex), pad = _object_shape(wl)
    py_a, px_a = (p * wl.step for p in period_scan_px)
    y = (np.arange(ey) - pad) * wl.dx
    x = (np.arange(ex) - pad) * wl.dx
    arg = np.zeros((ey, ex))
    if py_a:
        arg = arg + y[:, None] / py_a
    if px_a:
        arg = arg + x[None, :] / px_a
    return amp * np.cos(2 * math.pi * arg), pad


def vacuum_phase(wl: Workload) -> tuple:
    (ey, ex), pad = _object_shape(wl)
    return np.zeros((ey, ex)), pad


# ----------------------------------------------------------------------------------------------
# Frames and events


def _frame_batch_intensity(wl, phase_t, A_t, f0, f1, device, cdtype, rdtype):
    """Normalised probabilities p(k) for frames [f0, f1), shape (B, S*S), DC at (S/2, S/2)."""
    s = wl.sim
    ny, nx = wl.scan
    f = torch.arange(f0, f1, device=device)
    ry = torch.div(f, nx, rounding_mode="floor").to(rdtype)
    rx = (f % nx).to(rdtype)
    _, pad = _object_shape(wl)
    # probe centre in object pixels, then window origin (integer) and sub-pixel remainder
    cy = ry * (wl.step / wl.dx) + pad - s / 2.0
    cx = rx * (wl.step / wl.dx) + pad - s / 2.0
    oy = torch.floor(cy)
    ox = torch.floor(cx)
    dy = cy - oy + s / 2.0
    dx = cx - ox + s / 2.0
    kf = torch.fft.fftfreq(s, device=device, dtype=rdtype) * s
    ramp_y = torch.exp(torch.complex(torch.zeros_like(dy[:, None] * kf), -2 * math.pi * dy[:, None] * kf / s))
    ramp_x = torch.exp(torch.complex(torch.zeros_like(dx[:, None] * kf), -2 * math.pi * dx[:, None] * kf / s))
    spec = A_t[None] * ramp_y[:, :, None] * ramp_x[:, None, :]
    probe = torch.fft.ifft2(spec)
    iy = oy.long()[:, None] + torch.arange(s, device=device)[None]
    ix = ox.long()[:, None] + torch.arange(s, device=device)[None]
    win = phase_t[iy[:, :, None], ix[:, None, :]]
    trans = torch.exp(torch.complex(torch.zeros_like(win), win))
    psi = torch.fft.fft2(probe * trans.to(cdtype))
    inten = (psi.real * psi.real + psi.imag * psi.imag)
    inten = torch.fft.fftshift(inten, dim=(-2, -1)).reshape(inten.shape[0], -1)
    inten = torch.clamp(inten, min=0)
    return inten / inten.sum(dim=1, keepdim=True)


def simulate(wl: Workload, device="cpu", obj: str = "atoms", obj_args: dict | None = None,
             batch: int | None = None, noise_free: bool = False) -> EventData:
    """Simulate a whole acquisition and return its events.

    obj: "atoms" (default), "vacuum", "ramp" (obj_args g_px=(gy, gx)) or "cosine"
    (obj_args amp, period=(py, px) in scan steps).  With noise_free=True the
    per-frame probabilities are returned in meta["p"] (small workloads only).
    """
    obj_args = obj_args or {}
    if obj == "atoms":
        phase, pad = atoms_phase(wl)
    elif obj == "vacuum":
        phase, pad = vacuum_phase(wl)
    elif obj == "ramp":
        phase, pad = ramp_phase(wl, obj_args["g_px"])
    elif obj == "cosine":
        phase, pad = cosine_phase(wl, obj_args["amp"], obj_args["period"])
    else:
        raise ValueError(obj)
    device = torch.device(device)
    on_gpu = device.type != "cpu"
    rdtype = torch.float32 if on_gpu else torch.float64
    cdtype = torch.complex64 if on_gpu else torch.complex128
    phase_t = torch.as_tensor(phase, dtype=rdtype, device=device)
    A_t = torch.as_tensor(probe_spectrum(wl), dtype=cdtype, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(wl.event_seed)
    F = wl.n_frames
    s = wl.sim
    H, W = wl.det
    off_y, off_x = (H - s) // 2, (W - s) // 2
    if batch is None:
        batch = max(1, min(F, (1 << 27) // (s * s) if on_gpu else (1 << 21) // (s * s)))
    idx_parts, cnt_parts, p_parts = [], [], []
    for f0 in range(0, F, batch):
        f1 = min(F, f0 + batch)
        p = _frame_batch_intensity(wl, phase_t, A_t, f0, f1, device, cdtype, rdtype)
        if noise_free:
            p_parts.append(p.cpu().numpy())
        lam = torch.full((f1 - f0,), float(wl.mean_e), dtype=torch.float64, device=device)
        n_f = torch.poisson(lam, generator=gen).to(torch.int64)
        n_max = int(n_f.max().item()) if n_f.numel() else 0
        if n_max == 0:
            cnt_parts.append(n_f)
            continue
        draws = torch.multinomial(p, n_max, replacement=True, generator=gen)
        keep = torch.arange(n_max, device=device)[None, :] < n_f[:, None]
        sy = torch.div(draws, s, rounding_mode="floor") + off_y
        sx = draws % s + off_x
        k = sy * W + sx
        k = torch.where(keep, k, torch.full_like(k, H * W))
        k, _ = torch.sort(k, dim=1)
        idx_parts.append(k[keep].to(torch.int32))
        cnt_parts.append(n_f)
    counts = torch.cat(cnt_parts)
    off = torch.zeros(F + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(counts, 0)
    idx = torch.cat(idx_parts) if idx_parts else torch.zeros(0, dtype=torch.int32, device=device)
    meta = {"obj": obj, "obj_args": obj_args}
    if noise_free:
        meta["p"] = np.concatenate(p_parts)
    return EventData(wl, idx, off, phase, pad, meta)


# ----------------------------------------------------------------------------------------------
# Hand-made CSR inputs (edge cases and adversarial lists)


def random_csr(rng: np.random.Generator, n_frames: int, W: int, H: int, mean: float,
               p_empty: float = 0.1, sort: bool = True) -> tuple:
    """Uniform random hits, Poisson counts, some empty frames; duplicates allowed."""
    n = rng.poisson(mean, size=n_frames)
    n[rng.uniform(size=n_frames) < p_empty] = 0
    off = np.zeros(n_frames + 1, dtype=np.int64)
    off[1:] = np.cumsum(n)
    idx = rng.integers(0, W * H, size=int(off[-1])).astype(np.int32)
    if sort:
        for f in range(n_frames):
            idx[off[f]:off[f + 1]].sort()
    return idx, off


def with_pileup(idx: np.ndarray, off: np.ndarray, frame: int, pixel: int, count: int) -> tuple:
    """Insert `count` hits on one pixel into one frame (a coincidence pile-up)."""
    idx2 = np.concatenate([idx[:off[frame + 1]], np.full(count, pixel, np.int32), idx[off[frame + 1]:]])
    off2 = off.copy()
    off2[frame + 1:] += count
    return idx2.astype(np.int32), off2


def shuffle_within_frames(rng: np.random.Generator, idx: np.ndarray, off: np.ndarray) -> np.ndarray:
    out = idx.copy()
    for f in range(len(off) - 1):
        seg = out[off[f]:off[f + 1]]
        rng.shuffle(seg)
    return out


def run_length_form(idx, off):
    """Run-length form (Fig. 1c) of events sorted within their frames, as synthetic input for the
    re-coding path: d_0 = k_0 and d_i = k_i - k_(i-1) inside each frame (torch, same device)."""
    k = idx.to(torch.int64)
    d = k.clone()
    d[1:] -= k[:-1]
    starts = off[:-1][off[1:] > off[:-1]]  # first event of every non-empty frame
    d[starts] = k[starts]
    return d.to(torch.int32)
