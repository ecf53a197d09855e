"""Oracle: single-sideband (SSB) ptychography from a binned count cube (Sec. IV), FP64 numpy.

Test infrastructure only.  Steps, in the paper's order:

1. Scan-space transform (Eq. 2's left side): G(K, Q) = F_{R->Q} D(K, R), the
   unnormalised 2D DFT over the probe positions R = (ry, rx) of every kept
   detector pixel K, with numpy's sign exp(-2 pi i Q.R).
2. Double-overlap set (the pixel set defined after Eq. 2): for scan frequency Q,
   pixel K is used iff |K| < k0, |K - Q| < k0 and |K + Q| >= k0.  The printed
   set is garbled; this reading drops the A*(K+Q) sideband, which is what the text
   states the set is for.  Inside is strict '<', outside '>='.
3. Eq. 3: T(Q) = sum over K in the set of G(K, Q) / (A*(K) A(K - Q)).  With
   A = aperture * exp(-i chi), the divisor on the set is exp(i chi(K) - i chi(K - Q))
   and the sum is sum G exp(i (chi(K - Q) - chi(K))).  (The paper prints
   A(K) A*(K - Q), the complex conjugate of what Eq. 1 with numpy's FFT sign
   gives; this reading follows Eq. 1 and Eq. 2 and is pinned by an aberrated
   simulation.)  The sum is not divided by the number of pixels unless
   `normalize` is set; T(0) = 0 because the set is empty at Q = 0.
4. Phase image: phi = Im IFFT2(T) (numpy's 1/N normalisation).  For a weak phase
   object t(r) = i phi(r), so T is i phi~ weighted by the overlap count.

Units: K and Q are in unbinned detector pixels.  A scan frequency index m (numpy
fftfreq order, index N/2 -> -N/2) is Q = m * s with s = 1 / ((N * step) * dk)
pixels per index, evaluated exactly in that order.  Distances are evaluated as
(Kx - Qx)*(Kx - Qx) + (Ky - Qy)*(Ky - Qy) with each operation rounded (no fused
multiply-add), compared with r_bf * r_bf.

Aberration function (the paper only says the coefficients are tunable, Fig. 2):
the polynomial expansion in omega = lambda * k,
chi = (2 pi / lambda) [ C1 w^2/2 + A1a (wx^2 - wy^2)/2 + A1b wx wy + B2a w^2 wx/3 + B2b w^2 wy/3
                        + A2a (wx^3 - 3 wx wy^2)/3 + A2b (3 wx^2 wy - wy^3)/3 + C3 w^4/4 ],
coefficients in angstrom, order (C1, A1a, A1b, B2a, B2b, A2a, A2b, C3).  An optional
per-pixel probe phase theta[kd] enters as A(K) -> A(K) exp(-i theta(K)) on the
on-grid factor only, so the summand becomes G exp(i (chi(K - Q) - chi(K) - theta(K))).
"""
from __future__ import annotations

import math

import numpy as np

N_COEF = 8


def dft_matrix(n: int) -> np.ndarray:
    """W[m, r] = exp(-2 pi i ((m r) mod n) / n): the DFT with exact integer angle reduction."""
    m = np.arange(n, dtype=np.int64)
    return np.exp(-2j * math.pi * ((m[:, None] * m[None, :]) % n) / n)


def scan_dft_direct(D3: np.ndarray) -> np.ndarray:
    """G[kd] = W_y @ D[kd] @ W_x^T: the 2D DFT over (ry, rx) written as two matrix products."""
    n_k, ny, nx = D3.shape
    wy, wx = dft_matrix(ny), dft_matrix(nx)
    return np.matmul(np.matmul(wy[None], D3.astype(np.complex128)), wx.T[None])


def scan_dft(D3: np.ndarray) -> np.ndarray:
    """The same transform by numpy's FFT (FP64); checked against scan_dft_direct at small sizes."""
    return np.fft.fft2(D3.astype(np.float64), axes=(-2, -1))


def signed_freq_index(n: int) -> np.ndarray:
    """numpy fftfreq(n) * n as integers: 0, 1, ..., n/2 - 1, -n/2, ..., -1."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def q_scale(n: int, step: float, dk: float) -> float:
    """Detector pixels per scan-frequency index: 1 / ((n * step) * dk)."""
    return 1.0 / ((float(n) * step) * dk)


def chi(kx_px, ky_px, c, lam: float, dk: float):
    """Aberration phase chi at detector coordinates given in unbinned pixels."""
    c1, a1a, a1b, b2a, b2b, a2a, a2b, c3 = (float(v) for v in c)
    wx = lam * (np.asarray(kx_px) * dk)
    wy = lam * (np.asarray(ky_px) * dk)
    w2 = wx * wx + wy * wy
    poly = (0.5 * c1 * w2 + 0.5 * a1a * (wx * wx - wy * wy) + a1b * wx * wy
            + b2a * w2 * wx / 3.0 + b2b * w2 * wy / 3.0
            + a2a * (wx * wx * wx - 3.0 * wx * wy * wy) / 3.0
            + a2b * (3.0 * wx * wx * wy - wy * wy * wy) / 3.0
            + 0.25 * c3 * w2 * w2)
    return (2.0 * math.pi / lam) * poly


def chi_basis(kx_px, ky_px, lam: float, dk: float):
    """d chi / d c_j for the eight coefficients, as a list of arrays."""
    out = []
    for j in range(N_COEF):
        e = np.zeros(N_COEF)
        e[j] = 1.0
        out.append(chi(kx_px, ky_px, e, lam, dk))
    return out


def double_overlap(kx: float, ky: float, qx: np.ndarray, qy: np.ndarray, r2: float) -> np.ndarray:
    """Membership of pixel K in the double-overlap set of every Q (step 2 above)."""
    in_k = (kx * kx + ky * ky) < r2
    dx = kx - qx
    dy = ky - qy
    in_minus = (dx * dx + dy * dy) < r2
    ux = kx + qx
    uy = ky + qy
    out_plus = (ux * ux + uy * uy) >= r2
    return in_k & in_minus & out_plus


def scan_q_grid(ny: int, nx: int, step: float, dk: float):
    """(Qx, Qy) arrays of shape (Ny, Nx) in unbinned pixels, numpy fftfreq order."""
    sy, sx = q_scale(ny, step, dk), q_scale(nx, step, dk)
    qy = (signed_freq_index(ny).astype(np.float64) * sy)[:, None] * np.ones((1, nx))
    qx = (signed_freq_index(nx).astype(np.float64) * sx)[None, :] * np.ones((ny, 1))
    return qx, qy


def ssb_sum(G: np.ndarray, Kc: np.ndarray, step: float, dk: float, lam: float, r_bf: float,
            c=(0.0,) * N_COEF, theta=None, normalize: bool = False):
    """Eq. 3 over the double-overlap set.  G[kd, my, mx] full-spectrum scan transform.

    Returns (T[Ny, Nx] complex128, n_pairs[Ny, Nx] int64).
    """
    n_k, ny, nx = G.shape
    qx, qy = scan_q_grid(ny, nx, step, dk)
    r2 = float(r_bf) * float(r_bf)
    T = np.zeros((ny, nx), dtype=np.complex128)
    npair = np.zeros((ny, nx), dtype=np.int64)
    for kd in range(n_k):
        kx, ky = float(Kc[kd, 0]), float(Kc[kd, 1])
        m = double_overlap(kx, ky, qx, qy, r2)
        psi = chi(kx - qx, ky - qy, c, lam, dk) - chi(kx, ky, c, lam, dk)
        if theta is not None:
            psi = psi - float(theta[kd])
        T += np.where(m, G[kd] * np.exp(1j * psi), 0.0)
        npair += m
    if normalize:
        T = np.where(npair > 0, T / np.maximum(npair, 1), 0.0)
    return T, npair


def ssb_sum_bruteforce(G, Kc, step, dk, lam, r_bf, c=(0.0,) * N_COEF):
    """Eq. 3 as nested loops over Q and K (tiny inputs only)."""
    n_k, ny, nx = G.shape
    sy, sx = q_scale(ny, step, dk), q_scale(nx, step, dk)
    fy, fx = signed_freq_index(ny), signed_freq_index(nx)
    r2 = float(r_bf) * float(r_bf)
    T = np.zeros((ny, nx), dtype=np.complex128)
    for my in range(ny):
        for mx in range(nx):
            qx = float(fx[mx]) * sx
            qy = float(fy[my]) * sy
            acc = 0j
            for kd in range(n_k):
                kx, ky = float(Kc[kd, 0]), float(Kc[kd, 1])
                inside = kx * kx + ky * ky < r2
                dx, dy = kx - qx, ky - qy
                ux, uy = kx + qx, ky + qy
                if inside and dx * dx + dy * dy < r2 and ux * ux + uy * uy >= r2:
                    a_k = np.exp(-1j * chi(kx, ky, c, lam, dk))
                    a_kq = np.exp(-1j * chi(kx - qx, ky - qy, c, lam, dk))
                    acc += G[kd, my, mx] / (np.conj(a_k) * a_kq)
            T[my, mx] = acc
    return T


def g_panel(G: np.ndarray, lut: np.ndarray, qs) -> np.ndarray:
    """The scan transform at fixed scan frequencies as binned detector images (the panel of G
    at selected Q shown in Fig. 2): img[j, by, bx] = G[lut[by, bx], my_j, mx_j] for a kept bin,
    0 for a dropped one.  G is the full-spectrum cube G[kd, my, mx] of step 1; qs lists
    (my, mx) frequency indices in numpy fftfreq order, 0 <= my < Ny, 0 <= mx < Nx."""
    n_k, ny, nx = G.shape
    out = np.zeros((len(qs),) + lut.shape, dtype=np.complex128)
    kept = lut >= 0
    for j, (my, mx) in enumerate(qs):
        if not (0 <= my < ny and 0 <= mx < nx):
            raise ValueError("frequency index out of range")
        out[j][kept] = G[lut[kept], my, mx]
    return out


def phase_from_T(T: np.ndarray) -> np.ndarray:
    """phi = Im IFFT2(T) (step 4)."""
    return np.imag(np.fft.ifft2(T))


def cube(D: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """D[kd, f] with f = ry*Nx + rx -> D3[kd, ry, rx]."""
    return D.reshape(D.shape[0], ny, nx)


def ssb_forward(D: np.ndarray, Kc: np.ndarray, ny: int, nx: int, step: float, dk: float, lam: float,
                r_bf: float, c=(0.0,) * N_COEF, theta=None, normalize=False, direct=False):
    """D[kd, f] -> (phi, T, G)."""
    D3 = cube(D, ny, nx)
    G = scan_dft_direct(D3) if direct else scan_dft(D3)
    T, _ = ssb_sum(G, Kc, step, dk, lam, r_bf, c, theta, normalize)
    return phase_from_T(T), T, G


# ----------------------------------------------------------------------------------------------
# Loss and adjoint (not in the paper): L = -Var(phi) over all probe positions.


def neg_var_loss(phi: np.ndarray) -> float:
    """L = -(1/N_R) sum (phi - mean phi)^2 (population variance)."""
    d = phi - phi.mean()
    return -float(np.mean(d * d))


def neg_var_grad(phi: np.ndarray) -> np.ndarray:
    """dL/dphi = -(2/N_R) (phi - mean phi)."""
    return -(2.0 / phi.size) * (phi - phi.mean())


def ssb_adjoint(G: np.ndarray, Kc: np.ndarray, gbar: np.ndarray, step: float, dk: float, lam: float,
                r_bf: float, c=(0.0,) * N_COEF, theta=None):
    """Gradient of a loss L(phi) w.r.t. the 8 coefficients and the probe phase theta[kd].

    phi = Im IFFT2(T) gives dL/dRe T + i dL/dIm T = (i / N_R) FFT2(gbar) =: Tbar with
    gbar = dL/dphi.  Each summand of Eq. 3, z = G exp(i psi), moves with
    dz = i z dpsi, and dpsi/dc_j = B_j(K - Q) - B_j(K), dpsi/dtheta[kd] = -1, so
        dL/dc_j     = sum over pairs Re(conj(Tbar) i z) (B_j(K - Q) - B_j(K)),
        dL/dtheta_k = - sum over Q of Re(conj(Tbar) i z) for that pixel.
    """
    n_k, ny, nx = G.shape
    tbar = (1j / (ny * nx)) * np.fft.fft2(gbar)
    qx, qy = scan_q_grid(ny, nx, step, dk)
    r2 = float(r_bf) * float(r_bf)
    dc = np.zeros(N_COEF)
    dth = np.zeros(n_k)
    for kd in range(n_k):
        kx, ky = float(Kc[kd, 0]), float(Kc[kd, 1])
        m = double_overlap(kx, ky, qx, qy, r2)
        psi = chi(kx - qx, ky - qy, c, lam, dk) - chi(kx, ky, c, lam, dk)
        if theta is not None:
            psi = psi - float(theta[kd])
        w = np.where(m, np.real(np.conj(tbar) * 1j * G[kd] * np.exp(1j * psi)), 0.0)
        bm = chi_basis(kx - qx, ky - qy, lam, dk)
        bk = chi_basis(kx, ky, lam, dk)
        for j in range(N_COEF):
            dc[j] += float(np.sum(w * (bm[j] - bk[j])))
        dth[kd] = -float(np.sum(w))
    return dc, dth
