"""Oracle: centre-of-mass DPC phase integration (Sec. V), FP64 numpy.

Test infrastructure only.  Reading of the paper's update rule (its printed form
has no residual, no i or 2*pi factors and leaves lambda_1, lambda_2 and the
iteration count unset): gradient descent on || d_R phi - g ||^2 in Fourier space,

    Phi_{l+1}(q) = Phi_l(q) + mu * conj(D(q)) . (Ghat(q) - D(q) Phi_l(q))
                                  / (lambda_1 + |2 pi q|^2 + lambda_2 |2 pi q|^4)

with D(q) = 2 pi i q (numpy's FFT differentiates as multiplication by 2 pi i q),
Ghat the 2D FFT of the measured phase gradient g = 2 pi dk COM (rad/angstrom),
Phi_0 = 0, step size mu (0.5 in the paper).  The q = 0 term and the Nyquist
row/column of even-sized grids are held at zero.  phi = Re IFFT2(Phi_L).
"""
from __future__ import annotations

import math

import numpy as np


def com_to_gradient(com_x: np.ndarray, com_y: np.ndarray, dk: float):
    """Phase gradient from the centre of mass: grad phi = 2 pi <k> with <k> = dk * COM (Sec. V)."""
    return 2.0 * math.pi * dk * com_x, 2.0 * math.pi * dk * com_y


def dpc_integrate(gx: np.ndarray, gy: np.ndarray, step: float, mu: float = 0.5, lam1: float = 0.0,
                  lam2: float = 0.0, n_iter: int = 10) -> np.ndarray:
    """Regularised Fourier gradient descent for phi with d_R phi ~ (gx, gy) (Sec. V).

    gx, gy: (Ny, Nx) phase gradients in rad/angstrom on the scan grid of spacing `step`.
    """
    ny, nx = gx.shape
    Gx = np.fft.fft2(gx)
    Gy = np.fft.fft2(gy)
    qy = np.fft.fftfreq(ny, d=step)[:, None]
    qx = np.fft.fftfreq(nx, d=step)[None, :]
    Dx = 2j * math.pi * qx * np.ones((ny, 1))
    Dy = 2j * math.pi * qy * np.ones((1, nx))
    q2 = (2 * math.pi) ** 2 * (qx * qx + qy * qy)
    denom = lam1 + q2 + lam2 * q2 * q2
    live = denom != 0
    live[0, 0] = False
    if ny % 2 == 0:
        live[ny // 2, :] = False
    if nx % 2 == 0:
        live[:, nx // 2] = False
    safe = np.where(live, denom, 1.0)
    Phi = np.zeros((ny, nx), dtype=np.complex128)
    for _ in range(n_iter):
        rx = Gx - Dx * Phi
        ry = Gy - Dy * Phi
        step_dir = np.conj(Dx) * rx + np.conj(Dy) * ry
        Phi = np.where(live, Phi + mu * step_dir / safe, 0.0)
    return np.real(np.fft.ifft2(Phi))


def com_dpc(com_x: np.ndarray, com_y: np.ndarray, dk: float, step: float, **kw) -> np.ndarray:
    """COM image (detector px, shape (Ny, Nx)) -> DPC phase (Sec. V)."""
    gx, gy = com_to_gradient(com_x, com_y, dk)
    return dpc_integrate(gx, gy, step, **kw)
