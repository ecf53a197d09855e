"""Pins of the oracle's DPC integration (Sec. V) by closed forms on analytic phases."""
import math

import numpy as np
import pytest

from gen import WORKLOADS, probe_spectrum, simulate
from oracle import dpc, eer


def _cos_field(ny, nx, step, waves):
    """psi = sum a cos(2 pi (uy y + ux x) + p) with analytic gradient, on the scan grid."""
    y = (np.arange(ny) * step)[:, None]
    x = (np.arange(nx) * step)[None, :]
    psi = np.zeros((ny, nx))
    gx = np.zeros((ny, nx))
    gy = np.zeros((ny, nx))
    for a, my, mx, p in waves:
        uy, ux = my / (ny * step), mx / (nx * step)
        arg = 2 * math.pi * (uy * y + ux * x) + p
        psi += a * np.cos(arg)
        gx += -a * 2 * math.pi * ux * np.sin(arg)
        gy += -a * 2 * math.pi * uy * np.sin(arg)
    return psi, gx, gy


@pytest.mark.parametrize("n_iter", [1, 3, 10])
def test_gradient_of_bandlimited_phase_closed_form(n_iter):
    """P9: lambda1 = lambda2 = 0, g = grad psi -> phi_L = (1 - (1 - mu)^L) (psi - mean psi)."""
    ny, nx, step, mu = 24, 32, 0.2, 0.5
    psi, gx, gy = _cos_field(ny, nx, step, [(0.3, 1, 0, 0.1), (0.2, 3, -5, 1.0), (0.05, -7, 11, 2.0)])
    psi = psi + 0.7  # a constant is invisible to the gradient
    phi = dpc.dpc_integrate(gx, gy, step, mu=mu, n_iter=n_iter)
    expect = (1 - (1 - mu) ** n_iter) * (psi - psi.mean())
    assert np.max(np.abs(phi - expect)) < 1e-12


@pytest.mark.parametrize("lam1,lam2", [(0.5, 0.0), (0.0, 0.01), (2.0, 0.1)])
def test_regularised_single_wave_gain(lam1, lam2):
    """Per-frequency recurrence Phi <- Phi + mu (b - a Phi)/d has gain 1 - (1 - mu a/d)^L."""
    ny, nx, step, mu, L = 16, 16, 0.25, 0.5, 7
    my, mx = 2, 3
    psi, gx, gy = _cos_field(ny, nx, step, [(1.0, my, mx, 0.4)])
    q2 = (2 * math.pi) ** 2 * ((my / (ny * step)) ** 2 + (mx / (nx * step)) ** 2)
    d = lam1 + q2 + lam2 * q2 * q2
    gain = 1 - (1 - mu * q2 / d) ** L
    # a wave with gradient of gain... the least-squares target of grad psi is psi itself (scaled by q2/d)
    target = (q2 / d) * psi
    phi = dpc.dpc_integrate(gx, gy, step, mu=mu, lam1=lam1, lam2=lam2, n_iter=L)
    expect = (1 - (1 - mu * q2 / d) ** L) / (mu * q2 / d) * mu * target
    assert np.max(np.abs(phi - expect)) < 1e-12
    assert gain > 0


def test_nyquist_and_mean_are_removed():
    ny, nx, step = 8, 8, 0.2
    gx = np.cos(np.pi * np.arange(nx))[None, :] * np.ones((ny, 1))  # Nyquist along x
    phi = dpc.dpc_integrate(gx, np.zeros_like(gx), step, n_iter=5)
    assert np.max(np.abs(phi)) < 1e-14


@pytest.mark.parametrize("g", [(0, 3), (2, -1), (-4, 5)])
def test_com_gradient_scale_from_ramp_object(g):
    """Scale and sign of com_to_gradient (Sec. V: the DPC fit relates the phase gradient to the
    centre of mass, Eq. 4).  The generator's ramp object T = exp(i phi) with
    phi = 2 pi (g . dk) . r shifts the noise-free pattern by g pixels; events that are the
    shifted disk repeated evenly go through eer.com and com_to_gradient, and must give the slope
    of the generator's own phase array (rad per angstrom), independently of the oracle."""
    wl = WORKLOADS["small"].replace(scan=(2, 2))
    d = simulate(wl, obj="ramp", obj_args={"g_px": g}, noise_free=True)
    p = d.meta["p"]
    W, H = wl.det
    for f in range(p.shape[0]):
        # deterministic events: every pixel of the shifted disk 13 times (the disk is flat)
        reps = np.rint(p[f] * (13 * 793)).astype(np.int64)
        assert set(np.unique(reps)) == {0, 13}
        idx = np.repeat(np.arange(W * H), reps).astype(np.int32)
        off = np.array([0, len(idx)], dtype=np.int64)
        cx, cy, *_ = eer.com(idx, off, W, H)
        gx, gy = dpc.com_to_gradient(cx, cy, wl.dk)
        ph = d.phase_obj
        slope_x = (ph[0, 1] - ph[0, 0]) / wl.dx
        slope_y = (ph[1, 0] - ph[0, 0]) / wl.dx
        assert abs(gx[0] - slope_x) <= 1e-9 * max(abs(slope_x), 1e-3)
        assert abs(gy[0] - slope_y) <= 1e-9 * max(abs(slope_y), 1e-3)


@pytest.mark.parametrize("amp,period", [(0.02, (32, 0)), (0.02, (0, 16)), (0.05, (16, 16)), (0.3, (0, 32))])
def test_dpc_amplitude_equals_probe_intensity_transfer(amp, period):
    """Amplitude of the integrated DPC phase (Sec. V) for a cosine phase object.  For a pure
    phase object and a real (aberration-free) probe a, the centre of mass of each pattern is
    (1/2 pi) times the probe-intensity-weighted phase gradient, so the least-squares phase of
    the measured gradient is the object convolved with |a|^2 / sum |a|^2: a cosine of
    frequency u keeps its phase and has its amplitude scaled by H(u), the normalised Fourier
    transform of the probe intensity at u, computed here from the aperture alone.  With
    lambda1 = lambda2 = 0 and L iterations the integration gain is 1 - (1 - mu)^L.  A wrong
    factor anywhere between the pattern and the phase (2 pi, dk, the step) fails this."""
    wl = WORKLOADS["small"]
    d = simulate(wl, obj="cosine", obj_args={"amp": amp, "period": period}, noise_free=True)
    p = d.meta["p"]
    W, H = wl.det
    ky, kx = np.divmod(np.arange(W * H), W)
    comx = (p * (kx - W // 2)[None]).sum(1) / p.sum(1)
    comy = (p * (ky - H // 2)[None]).sum(1) / p.sum(1)
    ny, nx = wl.scan
    L, mu = 20, 0.5
    phi = dpc.com_dpc(comx.reshape(ny, nx), comy.reshape(ny, nx), wl.dk, wl.step, mu=mu, n_iter=L)
    y = (np.arange(ny) * wl.step)[:, None]
    x = (np.arange(nx) * wl.step)[None, :]
    uy = 1.0 / (period[0] * wl.step) if period[0] else 0.0
    ux = 1.0 / (period[1] * wl.step) if period[1] else 0.0
    arg = 2 * math.pi * (uy * y + ux * x)
    a_cos = 2 * np.mean(phi * np.cos(arg))
    a_sin = 2 * np.mean(phi * np.sin(arg))
    # H(u) from the aperture: probe a = IFFT(aperture), intensity on the simulation grid with
    # signed real-space coordinates (the probe is centred at r = 0)
    a = np.fft.ifft2(probe_spectrum(wl))
    inten = np.abs(a) ** 2
    f = np.fft.fftfreq(wl.sim) * wl.sim * wl.dx
    hu = float((inten * np.cos(2 * math.pi * (uy * f[:, None] + ux * f[None, :]))).sum() / inten.sum())
    expect = amp * hu * (1 - (1 - mu) ** L)
    assert 0.5 < hu < 1.0
    assert abs(a_cos - expect) <= 5e-3 * expect
    assert abs(a_sin) <= 1e-3 * expect
    # nothing at other frequencies beyond the simulation's own rounding
    resid = phi - a_cos * np.cos(arg)
    assert np.sqrt(np.mean(resid ** 2)) <= 1e-3 * expect


def test_dpc_recovers_object_from_noise_free_patterns():
    """P10 (approximate): noise-free COM of an atom field integrates to a phase that
    correlates with the probe-smoothed object."""
    wl = WORKLOADS["small"]
    d = simulate(wl, noise_free=True)
    p = d.meta["p"]
    W, H = wl.det
    ky, kx = np.divmod(np.arange(W * H), W)
    comx = (p * (kx - W // 2)[None]).sum(1) / p.sum(1)
    comy = (p * (ky - H // 2)[None]).sum(1) / p.sum(1)
    ny, nx = wl.scan
    phi = dpc.com_dpc(comx.reshape(ny, nx), comy.reshape(ny, nx), wl.dk, wl.step, n_iter=20)
    t = d.truth_at_scan()
    a, b = phi - phi.mean(), t - t.mean()
    assert (a * b).sum() / math.sqrt((a * a).sum() * (b * b).sum()) > 0.9
    # same pipeline from sampled events correlates too (weaker: shot noise)
    d2 = simulate(wl.replace(mean_e=3000.0))
    idx, off = d2.numpy()
    cx, cy, *_ = eer.com(idx, off, W, H)
    phi2 = dpc.com_dpc(cx.reshape(ny, nx), cy.reshape(ny, nx), wl.dk, wl.step)
    a = phi2 - phi2.mean()
    assert (a * b).sum() / math.sqrt((a * a).sum() * (b * b).sum()) > 0.6
