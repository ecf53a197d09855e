"""Pins of the oracle's scan transform, double-overlap sum, phase and adjoint (Sec. IV)."""
import math

import numpy as np
import pytest

from gen import C4_TRUE_ABERRATIONS, WORKLOADS, simulate
from oracle import eer, ssb


def _corr(a, b):
    a = a - a.mean()
    b = b - b.mean()
    return float((a * b).sum() / math.sqrt((a * a).sum() * (b * b).sum()))


# ----------------------------------------------------------------------------------------------
# scan transform


@pytest.mark.parametrize("shape", [(3, 8, 8), (2, 16, 4), (1, 5, 7)])
def test_fft_equals_direct_dft(shape):
    """P8: numpy's FFT (FP64) agrees with the exact-angle direct DFT."""
    rng = np.random.default_rng(0)
    D = rng.integers(0, 4, size=shape)
    a, b = ssb.scan_dft(D), ssb.scan_dft_direct(D)
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.abs(b).max())


def test_dc_equals_summed_pattern():
    """P6: G(K, Q=0) is the sum over probe positions of D(K, R), exactly (integer data)."""
    rng = np.random.default_rng(1)
    D = rng.integers(0, 9, size=(5, 32, 16))
    for G in (ssb.scan_dft(D), ssb.scan_dft_direct(D)):
        assert np.array_equal(G[:, 0, 0].real, D.sum(axis=(1, 2)).astype(np.float64))
        assert np.array_equal(G[:, 0, 0].imag, np.zeros(5))


def test_single_event_closed_form():
    """P7: D = delta(kd0, R0) gives G(kd0, Q) = exp(-2 pi i (my ry0/Ny + mx rx0/Nx))."""
    n_k, ny, nx, kd0, ry0, rx0 = 3, 8, 16, 1, 5, 11
    D = np.zeros((n_k, ny, nx))
    D[kd0, ry0, rx0] = 1
    my = np.arange(ny)[:, None]
    mx = np.arange(nx)[None, :]
    expect = np.exp(-2j * math.pi * (my * ry0 / ny + mx * rx0 / nx))
    for G in (ssb.scan_dft(D), ssb.scan_dft_direct(D)):
        assert np.max(np.abs(G[kd0] - expect)) < 1e-13
        assert np.max(np.abs(np.delete(G, kd0, axis=0))) == 0


def test_hermitian_and_parseval():
    """P8: real D gives G(K, -Q) = conj G(K, Q), and sum |G|^2 = N_R sum D^2."""
    rng = np.random.default_rng(2)
    D = rng.integers(0, 5, size=(4, 16, 8)).astype(np.float64)
    G = ssb.scan_dft(D)
    mirror = G[:, (-np.arange(16)) % 16][:, :, (-np.arange(8)) % 8]
    assert np.max(np.abs(mirror - np.conj(G))) < 1e-12
    assert abs((np.abs(G) ** 2).sum() - 128 * (D ** 2).sum()) < 1e-10 * (np.abs(G) ** 2).sum()


def test_g_panel_pins():
    """The panel of G at fixed Q: at Q = 0 it is the summed pattern of the events binned over
    bin x bin blocks on the kept bins (from the events, not from G); at -Q it is the conjugate
    of the panel at Q; a scan shifted by one position along x multiplies the panel at (my, mx)
    by exp(-2 pi i mx / Nx)."""
    wl = WORKLOADS["small"].replace(scan=(16, 8), bin=2, mean_e=30.0)
    d = simulate(wl, device="cpu")
    idx, off = d.numpy()
    H, W = wl.det
    ny, nx = wl.scan
    kc, lut = eer.bin_geometry(W, H, wl.bin, wl.r_bf)
    D = eer.bin_counts(idx, off, W, wl.bin, lut)
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    qs = [(0, 0), (3, 2), (ny - 3, nx - 2), (ny // 2, nx // 2), (1, nx - 1)]
    P = ssb.g_panel(G, lut, qs)
    assert P.shape == (len(qs), H // wl.bin, W // wl.bin)
    pac = eer.sum_frames(idx, off, W, H).reshape(H // wl.bin, wl.bin, W // wl.bin, wl.bin).sum(axis=(1, 3))
    assert np.array_equal(P[0].real, np.where(lut >= 0, pac, 0).astype(np.float64))
    assert np.all(P[0].imag == 0)
    assert np.all(P[:, lut < 0] == 0)
    assert np.max(np.abs(P[2] - np.conj(P[1]))) < 1e-9 * np.abs(P[1]).max()
    D3 = ssb.cube(D, ny, nx)
    Gs = ssb.scan_dft(np.roll(D3, 1, axis=2))
    Ps = ssb.g_panel(Gs, lut, qs)
    for j, (my, mx) in enumerate(qs):
        assert np.max(np.abs(Ps[j] - P[j] * np.exp(-2j * math.pi * mx / nx))) < 1e-9 * max(1.0, np.abs(P[j]).max())
    with pytest.raises(ValueError):
        ssb.g_panel(G, lut, [(ny, 0)])


def test_signed_frequency_index_and_scale():
    assert ssb.signed_freq_index(8).tolist() == [0, 1, 2, 3, -4, -3, -2, -1]
    assert ssb.q_scale(1024, 0.2, 0.5) == 1.0 / ((1024.0 * 0.2) * 0.5)


# ----------------------------------------------------------------------------------------------
# double-overlap sum (Eq. 3)


def _tiny_geometry():
    W = H = 16
    r_bf = 5.0
    kc, lut = eer.bin_geometry(W, H, 1, r_bf)
    return W, H, r_bf, kc, lut


def test_vectorised_sum_equals_nested_loops():
    """P12: the vectorised oracle equals Eq. 3 written as nested loops with the divisor A*(K)A(K-Q)."""
    W, H, r_bf, kc, lut = _tiny_geometry()
    rng = np.random.default_rng(3)
    ny, nx, step, lam = 8, 8, 0.2, 0.0196875
    dk = (0.025 / lam) / r_bf
    D = rng.integers(0, 3, size=(len(kc), ny * nx))
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    c = (40.0, 10.0, -15.0, 200.0, -100.0, 150.0, 80.0, 5e3)
    T, npair = ssb.ssb_sum(G, kc, step, dk, lam, r_bf, c)
    Tb = ssb.ssb_sum_bruteforce(G, kc, step, dk, lam, r_bf, c)
    assert npair.sum() > 0
    assert np.max(np.abs(T - Tb)) < 1e-10 * np.abs(Tb).max()


def test_normalised_sum_is_plain_sum_over_pair_count():
    """The normalised form of Eq. 3 (T divided by the size of the double-overlap set) against the
    nested-loop plain sum and a pair count by distances written out here: T_norm * n = T_plain
    where n > 0, and T_norm = 0 where the set is empty (Q = 0 among them)."""
    W, H, r_bf, kc, lut = _tiny_geometry()
    rng = np.random.default_rng(5)
    ny, nx, step, lam = 8, 12, 0.2, 0.0196875
    dk = (0.025 / lam) / r_bf
    D = rng.integers(0, 4, size=(len(kc), ny * nx))
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    c = (40.0, 10.0, -15.0, 200.0, -100.0, 150.0, 80.0, 5e3)
    Tn, _ = ssb.ssb_sum(G, kc, step, dk, lam, r_bf, c, normalize=True)
    Tb = ssb.ssb_sum_bruteforce(G, kc, step, dk, lam, r_bf, c)
    fy = np.rint(np.fft.fftfreq(ny) * ny)
    fx = np.rint(np.fft.fftfreq(nx) * nx)
    sy, sx = 1.0 / (ny * step * dk), 1.0 / (nx * step * dk)
    n = np.zeros((ny, nx), dtype=np.int64)
    for my in range(ny):
        for mx in range(nx):
            qx, qy = fx[mx] * sx, fy[my] * sy
            for kx, ky in kc:
                d_minus = math.hypot(kx - qx, ky - qy)
                d_plus = math.hypot(kx + qx, ky + qy)
                assert abs(d_minus - r_bf) > 1e-9 and abs(d_plus - r_bf) > 1e-9  # no ties here
                n[my, mx] += (math.hypot(kx, ky) < r_bf) and d_minus < r_bf and d_plus >= r_bf
    assert n[0, 0] == 0 and (n > 0).sum() > ny * nx // 2 and (n == 0).sum() > 1
    live = n > 0
    assert np.max(np.abs(Tn[live] * n[live] - Tb[live])) < 1e-10 * np.abs(Tb).max()
    assert np.all(Tn[~live] == 0)


def test_double_overlap_set_properties():
    W, H, r_bf, kc, lut = _tiny_geometry()
    ny, nx, step, lam = 8, 8, 0.2, 0.0196875
    dk = (0.025 / lam) / r_bf
    qx, qy = ssb.scan_q_grid(ny, nx, step, dk)
    r2 = r_bf * r_bf
    tot = np.zeros((ny, nx), dtype=np.int64)
    for kx, ky in kc:
        m = ssb.double_overlap(kx, ky, qx, qy, r2)
        assert not m[0, 0]  # empty at Q = 0, so T(0) = 0
        # independent restatement with distances: |K| < r, |K-Q| < r, |K+Q| >= r
        d1 = np.hypot(kx - qx, ky - qy)
        d2 = np.hypot(kx + qx, ky + qy)
        clear = (np.abs(d1 - r_bf) > 1e-9) & (np.abs(d2 - r_bf) > 1e-9)
        assert np.array_equal(m[clear], ((d1 < r_bf) & (d2 >= r_bf))[clear])
        tot += m
    # b = 1 keeps a set symmetric under K -> -K, so lune(Q) and lune(-Q) hold equally many pixels
    assert np.array_equal(tot, tot[(-np.arange(ny)) % ny][:, (-np.arange(nx)) % nx])


def test_vacuum_gives_zero_and_sum_is_linear():
    """P12: D constant over R puts all of G at Q = 0, where the set is empty, so T = 0; T is linear in D."""
    W, H, r_bf, kc, lut = _tiny_geometry()
    ny, nx, step, lam = 8, 8, 0.2, 0.0196875
    dk = (0.025 / lam) / r_bf
    c = C4_TRUE_ABERRATIONS
    D = np.repeat(np.arange(1, len(kc) + 1)[:, None], ny * nx, axis=1)
    _, T, _ = ssb.ssb_forward(D, kc, ny, nx, step, dk, lam, r_bf, c)
    assert np.max(np.abs(T)) < 1e-9
    rng = np.random.default_rng(4)
    D1 = rng.integers(0, 4, size=D.shape)
    D2 = rng.integers(0, 4, size=D.shape)
    _, T1, _ = ssb.ssb_forward(D1, kc, ny, nx, step, dk, lam, r_bf, c)
    _, T2, _ = ssb.ssb_forward(D2, kc, ny, nx, step, dk, lam, r_bf, c)
    _, T12, _ = ssb.ssb_forward(3 * D1 + D2, kc, ny, nx, step, dk, lam, r_bf, c)
    assert np.max(np.abs(T12 - 3 * T1 - T2)) < 1e-9 * np.abs(T12).max()


def _noise_free_D(wl, p, kc, lut):
    H, W = wl.det
    b = wl.bin
    blocks = p.reshape(p.shape[0], H // b, b, W // b, b).sum(axis=(2, 4))
    D = np.zeros((len(kc), p.shape[0]))
    by, bx = np.nonzero(lut >= 0)
    D[lut[by, bx]] = blocks[:, by, bx].T
    return D


def test_weak_cosine_object_is_recovered():
    """P13 (approximate): noise-free weak cosine, chi = 0: the SSB phase follows the object."""
    wl = WORKLOADS["small"]
    d = simulate(wl, obj="cosine", obj_args={"amp": 0.01, "period": (0, 5)}, noise_free=True)
    kc, lut = eer.bin_geometry(wl.det[1], wl.det[0], wl.bin, wl.r_bf)
    D = _noise_free_D(wl, d.meta["p"], kc, lut)
    phi, T, G = ssb.ssb_forward(D, kc, *wl.scan, wl.step, wl.dk, wl.lam, wl.r_bf)
    assert _corr(phi, d.truth_at_scan()) > 0.93


def test_aberration_convention_pinned_by_simulation():
    """P11: data simulated with an aberrated probe is recovered with the same coefficients;
    zero coefficients, or the conjugate divisor printed in Eq. 3, do much worse."""
    wl = WORKLOADS["small"].replace(aberr=C4_TRUE_ABERRATIONS)
    d = simulate(wl, noise_free=True)
    kc, lut = eer.bin_geometry(wl.det[1], wl.det[0], wl.bin, wl.r_bf)
    D = _noise_free_D(wl, d.meta["p"], kc, lut)
    truth = d.truth_at_scan()
    ny, nx = wl.scan
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    T_true, npair = ssb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf, wl.aberr)
    T_zero, _ = ssb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf)
    # the literal printed divisor A(K)A*(K-Q) flips the sign of psi: same as coefficients -c
    T_conj, _ = ssb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf, tuple(-v for v in wl.aberr))
    filt = np.real(np.fft.ifft2(np.fft.fft2(truth) * npair))
    c_true = _corr(ssb.phase_from_T(T_true), filt)
    assert c_true > 0.85
    assert _corr(ssb.phase_from_T(T_zero), filt) < c_true - 0.4
    assert _corr(ssb.phase_from_T(T_conj), filt) < c_true - 0.4
    # the unaberrated reference pair reaches a similar correlation
    wl0 = WORKLOADS["small"]
    d0 = simulate(wl0, noise_free=True)
    D0 = _noise_free_D(wl0, d0.meta["p"], kc, lut)
    phi0, _, _ = ssb.ssb_forward(D0, kc, ny, nx, wl0.step, wl0.dk, wl0.lam, wl0.r_bf)
    assert abs(_corr(phi0, filt) - c_true) < 0.1


# ----------------------------------------------------------------------------------------------
# adjoint


def test_adjoint_matches_central_differences():
    """P14: dL/dc and dL/dtheta of L = -Var(phi) equal central finite differences."""
    W, H, r_bf, kc, lut = _tiny_geometry()
    rng = np.random.default_rng(5)
    ny, nx, step, lam = 8, 8, 0.2, 0.0196875
    dk = (0.025 / lam) / r_bf
    D = rng.integers(0, 4, size=(len(kc), ny * nx))
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    c = np.array(C4_TRUE_ABERRATIONS) * (1 + rng.uniform(-0.5, 0.5, size=8))
    theta = rng.uniform(-0.3, 0.3, size=len(kc))

    def loss(cc, th):
        T, _ = ssb.ssb_sum(G, kc, step, dk, lam, r_bf, cc, th)
        return ssb.neg_var_loss(ssb.phase_from_T(T))

    T, _ = ssb.ssb_sum(G, kc, step, dk, lam, r_bf, c, theta)
    gbar = ssb.neg_var_grad(ssb.phase_from_T(T))
    dc, dth = ssb.ssb_adjoint(G, kc, gbar, step, dk, lam, r_bf, c, theta)
    for j in range(8):
        h = 1e-6 * max(abs(c[j]), 1.0)
        e = np.zeros(8)
        e[j] = h
        fd = (loss(c + e, theta) - loss(c - e, theta)) / (2 * h)
        assert abs(dc[j] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(dc).max())
    for kd in [0, 7, len(kc) // 2, len(kc) - 1]:
        e = np.zeros(len(kc))
        e[kd] = 1e-6
        fd = (loss(c, theta + e) - loss(c, theta - e)) / 2e-6
        assert abs(dth[kd] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(dth).max())


def test_loss_gradient_formula():
    rng = np.random.default_rng(6)
    phi = rng.normal(size=(4, 6))
    g = ssb.neg_var_grad(phi)
    for _ in range(3):
        i, j = rng.integers(0, 4), rng.integers(0, 6)
        e = np.zeros_like(phi)
        e[i, j] = 1e-6
        fd = (ssb.neg_var_loss(phi + e) - ssb.neg_var_loss(phi - e)) / 2e-6
        assert abs(g[i, j] - fd) < 1e-8


@pytest.mark.parametrize("j", range(8))
def test_each_aberration_term_pinned_by_simulation(j):
    """P11 per coefficient: a probe carrying only c_j (about 3 rad at the disk edge) is
    recovered best with +c_j, against 0 and -c_j (catches a wrong sign, factor or term in chi)."""
    base = WORKLOADS["small"]
    omega = base.lam * base.k0
    powers = [2, 2, 2, 3, 3, 3, 3, 4]
    scale = [0.5, 0.5, 1.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 0.25]
    cj = 3.0 / ((2 * math.pi / base.lam) * scale[j] * omega ** powers[j])
    ab = [0.0] * 8
    ab[j] = cj
    wl = base.replace(aberr=tuple(ab), scan=(24, 24))
    d = simulate(wl, noise_free=True)
    kc, lut = eer.bin_geometry(wl.det[1], wl.det[0], wl.bin, wl.r_bf)
    D = _noise_free_D(wl, d.meta["p"], kc, lut)
    ny, nx = wl.scan
    G = ssb.scan_dft(ssb.cube(D, ny, nx))
    truth = d.truth_at_scan()
    scores, var = {}, {}
    for sgn in (1.0, 0.0, -1.0):
        c = [0.0] * 8
        c[j] = sgn * cj
        T, npair = ssb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf, c)
        filt = np.real(np.fft.ifft2(np.fft.fft2(truth) * npair))
        phi = ssb.phase_from_T(T)
        scores[sgn] = _corr(phi, filt)
        var[sgn] = float(phi.var())
    # the right coefficient sums the sideband coherently: largest phase variance
    assert var[0.0] < 0.9 * var[1.0] and var[-1.0] < 0.6 * var[1.0]
    assert scores[1.0] > 0.8 and scores[1.0] > scores[-1.0] + 0.1
