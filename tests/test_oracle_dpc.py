"""Pins of the oracle's DPC integration (Sec. V) by closed forms on analytic phases."""
import math

import numpy as np
import pytest

from gen import WORKLOADS, simulate
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


def test_com_gradient_sign_from_ramp():
    """COM of a phase ramp of slope 2 pi g is g: com_to_gradient returns 2 pi g dk (rad/A)."""
    gx, gy = dpc.com_to_gradient(np.array([3.0]), np.array([-1.0]), 0.05)
    assert gx[0] == pytest.approx(2 * math.pi * 0.15) and gy[0] == pytest.approx(-2 * math.pi * 0.05)


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
