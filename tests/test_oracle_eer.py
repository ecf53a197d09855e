"""Pins of the oracle's event reductions: counts, centre of mass, binning (Table 1, Eq. 4)."""
import math
import os

import numpy as np
import pytest

from gen import WORKLOADS, random_csr, shuffle_within_frames, simulate, with_pileup
from oracle import eer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            out[key.strip()] = [float(v) for v in val.split()]
    return out


def test_hand_worked_example():
    g = _read_golden("eer_hand.txt")
    W, H = int(g["W"][0]), int(g["H"][0])
    idx = np.array(g["idx"], dtype=np.int32)
    off = np.array(g["off"], dtype=np.int64)
    cx_, cy_, sx, sy, n = eer.com(idx, off, W, H)
    assert n.tolist() == [int(v) for v in g["counts"]]
    assert sx.tolist() == [int(v) for v in g["sx"]]
    assert sy.tolist() == [int(v) for v in g["sy"]]
    assert cx_.tolist() == g["com_x"]
    assert cy_.tolist() == g["com_y"]
    kc, lut = eer.bin_geometry(W, H, int(g["bin"][0]), g["r_bf"][0])
    assert kc.ravel().tolist() == g["kc"]
    D = eer.bin_counts(idx, off, W, int(g["bin"][0]), lut)
    assert D.ravel().tolist() == [int(v) for v in g["D"]]


@pytest.mark.parametrize("seed", range(6))
def test_counts_and_com_match_dense_bruteforce(seed):
    """P1, P2: event-based counts and COM equal the dense-frame computation exactly."""
    rng = np.random.default_rng(seed)
    W, H = [(8, 8), (6, 10), (16, 4)][seed % 3]
    idx, off = random_csr(rng, 40, W, H, mean=5.0, p_empty=0.2, sort=seed % 2 == 0)
    if seed >= 3:
        idx, off = with_pileup(idx, off, 7, W * H - 1, 30)
        idx = shuffle_within_frames(rng, idx, off)
    rho = eer.dense_frames(idx, off, W, H)
    n = eer.frame_counts(off)
    assert (rho.sum(axis=(1, 2)) == n).all()
    assert n.sum() == len(idx)
    for cx, cy in [(W // 2, H // 2), (0, 0), (W - 1, 1)]:
        a = eer.com(idx, off, W, H, cx, cy)
        b = eer.com_dense(rho, cx, cy)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_com_empty_frames_are_zero():
    idx = np.array([3, 3], dtype=np.int32)
    off = np.array([0, 0, 2, 2], dtype=np.int64)
    cx, cy, _, _, n = eer.com(idx, off, 4, 4)
    assert n.tolist() == [0, 2, 0]
    assert cx.tolist() == [0.0, 1.0, 0.0] and cy.tolist() == [0.0, -2.0, 0.0]


def test_symmetric_disk_com_is_zero():
    """P4: the integer points of a disk about the zero-frequency pixel have COM exactly 0."""
    W = H = 64
    k = [ky * W + kx for ky in range(H) for kx in range(W) if (kx - 32) ** 2 + (ky - 32) ** 2 < 16 ** 2]
    idx = np.array(k, dtype=np.int32)
    off = np.array([0, len(k)], dtype=np.int64)
    cx, cy, sx, sy, n = eer.com(idx, off, W, H)
    assert sx[0] == 0 and sy[0] == 0 and cx[0] == 0.0 and cy[0] == 0.0
    # lattice points strictly inside r = 16, counted column by column
    r2 = 256
    count = sum(2 * math.isqrt(r2 - 1 - x * x) + 1 for x in range(-15, 16))
    assert n[0] == count == 793


@pytest.mark.parametrize("g", [(0, 3), (2, -1), (-4, 5)])
def test_phase_ramp_shifts_com_exactly(g):
    """P3: T = exp(2 pi i g.r) shifts the noise-free pattern by g pixels; its COM is g exactly."""
    wl = WORKLOADS["small"].replace(scan=(2, 3))
    d = simulate(wl, obj="ramp", obj_args={"g_px": g}, noise_free=True)
    p = d.meta["p"]
    W, H = wl.det
    for f in range(p.shape[0]):
        on = np.nonzero(p[f] > 0.5 * p[f].max())[0]  # the shifted bright-field disk
        idx = on.astype(np.int32)
        off = np.array([0, len(idx)], dtype=np.int64)
        cx, cy, _, _, n = eer.com(idx, off, W, H)
        assert n[0] == 793
        assert (cy[0], cx[0]) == (float(g[0]), float(g[1]))


def test_phase_ramp_poisson_com_within_noise():
    """P3 with Poisson sampling: mean COM over frames matches g within 5 standard errors."""
    wl = WORKLOADS["small"].replace(scan=(8, 8), mean_e=50.0)
    g = (1, 2)
    d = simulate(wl, obj="ramp", obj_args={"g_px": g})
    idx, off = d.numpy()
    W, H = wl.det
    cx, cy, _, _, n = eer.com(idx, off, W, H)
    var1 = 16.0 ** 2 / 4.0  # per-axis variance of a uniform disk of radius 16
    se = math.sqrt(var1 / n.sum())
    assert abs(np.sum(cx * n) / n.sum() - g[1]) < 5 * se
    assert abs(np.sum(cy * n) / n.sum() - g[0]) < 5 * se


@pytest.mark.parametrize("b,W,H,r", [(1, 8, 8, 3.0), (2, 8, 12, 3.5), (3, 12, 9, 4.0), (4, 16, 16, 6.0)])
def test_binning_matches_dense_bruteforce(b, W, H, r):
    """P1, P5: event binning/cropping equals block sums of dense frames; kept sums <= N_f."""
    rng = np.random.default_rng(b)
    idx, off = random_csr(rng, 30, W, H, mean=8.0)
    kc, lut = eer.bin_geometry(W, H, b, r)
    D = eer.bin_counts(idx, off, W, b, lut)
    Dd = eer.bin_dense(eer.dense_frames(idx, off, W, H), b, lut)
    assert np.array_equal(D, Dd)
    n = eer.frame_counts(off)
    assert (D.sum(axis=0) <= n).all()
    # equality iff every event of the frame lands in a kept bin
    k = idx.astype(np.int64)
    inside = lut[(k // W) // b, (k % W) // b] >= 0
    f = eer.frame_of_event(off)
    n_in = np.bincount(f[inside], minlength=len(n))
    assert np.array_equal(D.sum(axis=0), n_in)


def test_bin_geometry_kept_set():
    """Kept bins are exactly those with half-integer centre strictly inside the disk."""
    for W, b, r, n_expect in [(64, 1, 16.0, 793), (576, 8, 60.0, None), (576, 4, 60.0, None),
                              (576, 6, 60.0, None)]:
        kc, lut = eer.bin_geometry(W, W, b, r)
        # independent count: centres b*j + (b-1)/2 - W/2 along each axis
        cen = np.array([b * j + (b - 1) / 2.0 - W / 2 for j in range(W // b)])
        cnt = int(((cen[:, None] ** 2 + cen[None, :] ** 2) < r * r).sum())
        assert len(kc) == cnt == (lut >= 0).sum()
        if n_expect:
            assert cnt == n_expect
        assert (np.diff(lut[lut >= 0]) == 1).all()  # raster numbering


def test_generator_counts_are_poisson_and_inside_detector():
    wl = WORKLOADS["small"]
    d = simulate(wl)
    idx, off = d.numpy()
    n = eer.frame_counts(off)
    assert off[0] == 0 and off[-1] == len(idx) and (n >= 0).all()
    assert abs(n.mean() - wl.mean_e) < 5 * math.sqrt(wl.mean_e / len(n))
    assert idx.min() >= 0 and idx.max() < wl.det[0] * wl.det[1]
    for f in range(0, len(n), 97):
        seg = idx[off[f]:off[f + 1]]
        assert (np.diff(seg) >= 0).all()


# ----------------------------------------------------------------------------------------------
# virtual detectors: radial sums and frame sums (Table 1)


def test_radial_sum_and_frame_sum_hand_example():
    g = _read_golden("eer_hand.txt")
    W, H = int(g["W"][0]), int(g["H"][0])
    idx = np.array(g["idx"], dtype=np.int32)
    off = np.array(g["off"], dtype=np.int64)
    rs = eer.radial_sum(idx, off, W, H, g["radial_in"], g["radial_out"])
    assert rs[0].tolist() == [int(v) for v in g["radial_A"]]
    assert rs[1].tolist() == [int(v) for v in g["radial_B"]]
    assert eer.sum_frames(idx, off, W, H).ravel().tolist() == [int(v) for v in g["sum"]]


def test_radial_sum_brute_force_dense():
    """Pixel loops over dense frames (the dense-format column of Table 1)."""
    rng = np.random.default_rng(21)
    W, H = 11, 9
    idx, off = random_csr(rng, 30, W, H, 12.0)
    rho = eer.dense_frames(idx, off, W, H)
    cx, cy = W // 2, H // 2
    r_in, r_out = [0.0, 1.0, 2.5, 3.0], [1.0, 2.5, 3.0, 100.0]
    got = eer.radial_sum(idx, off, W, H, r_in, r_out)
    for j, (a, b) in enumerate(zip(r_in, r_out)):
        for f in range(len(off) - 1):
            tot = 0
            for ky in range(H):
                for kx in range(W):
                    d2 = (kx - cx) ** 2 + (ky - cy) ** 2
                    if a * a <= d2 < b * b:
                        tot += int(rho[f, ky, kx])
            assert got[j, f] == tot


def test_radial_sum_special_cases():
    rng = np.random.default_rng(22)
    W, H = 16, 16
    idx, off = random_csr(rng, 50, W, H, 20.0)
    # the whole detector: every event, N_f
    assert np.array_equal(eer.radial_sum(idx, off, W, H, [0.0], [1e9])[0], eer.frame_counts(off))
    # additivity of adjacent annuli
    a = eer.radial_sum(idx, off, W, H, [1.0, 3.5], [3.5, 6.0])
    b = eer.radial_sum(idx, off, W, H, [1.0], [6.0])
    assert np.array_equal(a.sum(axis=0), b[0])
    # an empty annulus
    assert not eer.radial_sum(idx, off, W, H, [2.0], [2.0]).any()


def test_frame_sum_brute_force_and_ranges():
    rng = np.random.default_rng(23)
    W, H = 10, 7
    idx, off = random_csr(rng, 40, W, H, 9.0)
    rho = eer.dense_frames(idx, off, W, H)
    assert np.array_equal(eer.sum_frames(idx, off, W, H), rho.sum(axis=0))
    assert np.array_equal(eer.sum_frames(idx, off, W, H, 5, 20), rho[5:25].sum(axis=0))
    assert eer.sum_frames(idx, off, W, H, 5, 20).sum() == off[25] - off[5]
    left = eer.sum_frames(idx, off, W, H, 0, 17)
    right = eer.sum_frames(idx, off, W, H, 17, 23)
    assert np.array_equal(left + right, eer.sum_frames(idx, off, W, H))


# ----------------------------------------------------------------------------------------------
# run-length form (Fig. 1c) and its re-coding to linear indices


def test_rle_hand_example():
    g = _read_golden("eer_hand.txt")
    idx = np.array(g["idx"], dtype=np.int32)
    off = np.array(g["off"], dtype=np.int64)
    d = eer.rle_encode(idx, off)
    assert d.tolist() == [int(v) for v in g["rle"]]
    assert eer.rle_decode(d, off).tolist() == [int(v) for v in g["idx_sorted"]]


def test_rle_round_trip_and_invariants():
    rng = np.random.default_rng(41)
    W, H = 30, 20
    idx, off = random_csr(rng, 400, W, H, 15.0, sort=False)
    d = eer.rle_encode(idx, off)
    assert (d >= 0).all()
    k = eer.rle_decode(d, off)
    for f in range(len(off) - 1):
        seg = slice(off[f], off[f + 1])
        assert np.array_equal(k[seg], np.sort(idx[seg]))
        if off[f + 1] > off[f]:
            # the distances of a frame add up to its largest index
            assert d[seg].sum() == idx[seg].max()
    # decoding a sorted list and re-encoding it is the identity
    assert np.array_equal(eer.rle_encode(k, off), d)
    # the reductions see the same events
    assert np.array_equal(eer.com(k, off, W, H)[4], eer.com(idx, off, W, H)[4])
    assert np.array_equal(eer.sum_frames(k, off, W, H), eer.sum_frames(idx, off, W, H))


def test_generator_run_length_form_matches_oracle():
    """The benchmark's synthetic run-length input equals the oracle's encoding of sorted frames."""
    import torch
    from gen import run_length_form

    rng = np.random.default_rng(52)
    idx, off = random_csr(rng, 300, 25, 17, 12.0, p_empty=0.2, sort=True)
    got = run_length_form(torch.from_numpy(idx), torch.from_numpy(off)).numpy()
    assert np.array_equal(got, eer.rle_encode(idx, off))
