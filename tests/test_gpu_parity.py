"""GPU parity of the HIP path against the FP64 oracle (small sizes: full element-by-element).

Integer work (counts, binned cube, G(K, 0)) is compared bit for bit; FP32 outputs by
relative L2 against the oracle with the tolerance 1e-5.
"""
import numpy as np
import pytest
import torch

import paper_2104_06336_amd as stem
from gen import C4_TRUE_ABERRATIONS, WORKLOADS, random_csr, shuffle_within_frames, simulate, with_pileup
from oracle import eer as oeer
from oracle import ssb as ossb

from helpers import (gpu_com, gpu_ssb, oracle_dpc, oracle_pruned, oracle_row_dft, oracle_ssb, per_q_error,
                     q_error_scale, rel_l2, state_D, state_kc, state_npair, state_pruned, state_X, structs, to_device)

pytestmark = pytest.mark.gpu

TOL = 1e-5

SMALL = WORKLOADS["small"]
# 576x576 detector binned 8x on a 64x64 scan (the large workloads' pixel set, oracle-sized)
MID = WORKLOADS["scan1024"].replace(name="mid: scan 64x64, 576 detector binned 8x", scan=(64, 64))
# non-square scan, binning 2 of a 64x64 detector
RECT = SMALL.replace(name="rect: scan 32x64, binned 2x", scan=(32, 64), bin=2, mean_e=30.0)
ABERR = SMALL.replace(name="small aberrated", aberr=C4_TRUE_ABERRATIONS)
# other transform lengths: 128 (FFT radix plan 16.8, matrix-core blocks of 4) and 512 x 256
# (plans 16.16.2 / 16.16, blocks of 16 and 8), aberrated
N128 = SMALL.replace(name="scan 128x128", scan=(128, 128), aberr=C4_TRUE_ABERRATIONS)
N512 = SMALL.replace(name="scan 512x256, binned 2x", scan=(512, 256), bin=2, mean_e=10.0)

# 1024-point column transform (plan 16.16.4) on a tall, narrow scan
N1024 = SMALL.replace(name="scan 1024x32", scan=(1024, 32), mean_e=15.0)
# unbinned wide disk: about 4600 bins in the kept set's bounding box, more than the binning kernel's
# LDS table holds, so pixels are mapped through the global per-pixel table
WIDE = SMALL.replace(name="wide disk: detector 192x192 unbinned, r_bf 34 px", det=(192, 192), r_bf=34.0,
                     sim=192, mean_e=60.0)

CASES = {"small": SMALL, "mid": MID, "rect": RECT, "aberr": ABERR, "n128": N128, "n512": N512, "n1024": N1024,
         "wide": WIDE}
_DATA = {}


def data(name):
    if name not in _DATA:
        wl = CASES[name]
        d = simulate(wl, device="cuda" if wl.n_frames > 8192 else "cpu")
        idx, off = d.numpy()
        _DATA[name] = (wl, idx, off)
    return _DATA[name]


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)


# ----------------------------------------------------------------------------------------------
# centre of mass and DPC


@pytest.mark.parametrize("name", ["small", "mid", "rect", "n512"])
def test_com_bit_exact(gpu, name):
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    g = gpu_com(d_idx, d_off, wl)
    H, W = wl.det
    cx, cy, sx, sy, n = oeer.com(idx, off, W, H)
    assert g["status"] == 0
    assert np.array_equal(g["counts"], n)
    assert np.array_equal(g["com64"][0], cx) and np.array_equal(g["com64"][1], cy)
    assert np.array_equal(g["com32"][0], cx.astype(np.float32))
    assert np.array_equal(g["com32"][1], cy.astype(np.float32))


def test_com_chunks_and_edge_frames(gpu):
    """Empty frames, a 300-event pile-up, unsorted frames; four chunks equal one call."""
    rng = np.random.default_rng(11)
    wl = SMALL.replace(scan=(32, 33))  # F = 1056: ragged last block of frames
    idx, off = random_csr(rng, wl.n_frames, 64, 64, mean=20.0, p_empty=0.3)
    idx, off = with_pileup(idx, off, 17, 64 * 31 + 5, 300)
    idx = shuffle_within_frames(rng, idx, off)
    d_idx, d_off = to_device(idx, off)
    det, scan, optics = structs(wl)
    F = wl.n_frames
    com64 = torch.zeros(2 * F, dtype=torch.float64, device="cuda")
    st = stem.status_tensor()
    for f0 in range(0, F, 300):
        stem.com_dpc(d_idx, d_off, f0, min(300, F - f0), det, scan, com64=com64, d_status=st)
    cx, cy, *_ = oeer.com(idx, off, 64, 64)
    c = com64.cpu().numpy().reshape(2, F)
    assert int(st.item()) == 0
    assert np.array_equal(c[0], cx) and np.array_equal(c[1], cy)


@pytest.mark.parametrize("name", ["small", "mid", "rect"])
@pytest.mark.parametrize("reg", [(0.0, 0.0, 10), (1.0, 0.05, 25)])
def test_dpc_phase_parity(gpu, name, reg):
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    lam1, lam2, L = reg
    g = gpu_com(d_idx, d_off, wl, phase=True, dpc_params=stem.Dpc(0.5, lam1, lam2, L))
    ref = oracle_dpc(idx, off, wl, lam1=lam1, lam2=lam2, n_iter=L)
    assert g["status"] == 0
    assert rel_l2(g["phase"], ref) <= TOL


# ----------------------------------------------------------------------------------------------
# binning, scan transform, sideband sum, phase


@pytest.mark.parametrize("name", ["small", "mid", "rect", "n128", "n512", "wide"])
def test_binning_and_scan_transform(gpu, name):
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl)
    ref = oracle_ssb(idx, off, wl)
    assert out["status"] == 0
    assert np.array_equal(state_kc(st), ref["kc"])
    assert np.array_equal(state_D(st, wl), ref["D"])
    # the row transform of every pixel, and its zero-frequency column: the row sums, exactly
    X = state_X(st, wl)
    assert rel_l2(X, oracle_row_dft(ref["D"], wl)) <= TOL
    rows = ossb.cube(ref["D"], *wl.scan).sum(axis=2)
    assert np.array_equal(X[:, :, 0].real.astype(np.float64), rows.astype(np.float64))
    assert np.all(X[:, :, 0].imag == 0)
    # G on the double-overlap pairs: every (pixel, column) run has the oracle's length (the sets
    # are equal pair by pair) and the values match
    pg, poff = state_pruned(st)
    pg_ref, poff_ref = oracle_pruned(ref["G"], ref["kc"], wl)
    assert np.array_equal(poff, poff_ref)
    assert rel_l2(pg, pg_ref) <= TOL


@pytest.mark.parametrize("name", ["small", "mid", "rect", "aberr", "n128", "n512", "n1024"])
def test_ssb_phase_parity(gpu, name):
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    c = wl.aberr
    theta = None
    if name == "aberr":
        det, _, optics = structs(wl)
        theta = np.random.default_rng(3).uniform(-0.3, 0.3, size=stem.ssb_num_pixels(det, optics))
    st, out = gpu_ssb(d_idx, d_off, wl, c=c, theta=theta)
    ref = oracle_ssb(idx, off, wl, c=c, theta=None if theta is None else theta.astype(np.float32))
    assert out["status"] == 0
    assert rel_l2(out["T"], ref["T"]) <= TOL
    assert rel_l2(out["phi"], ref["phi"]) <= TOL
    assert out["T"][0, 0] == 0
    # every Q, relative to its own summands
    assert per_q_error(out["T"], ref["T"], q_error_scale(ref["G"], ref["kc"], wl)) <= 1e-4


def test_ssb_normalized_parity(gpu):
    wl, idx, off = data("small")
    d_idx, d_off = to_device(idx, off)
    for g_mode in (stem.STEM_G_STORE, stem.STEM_G_RECOMPUTE):
        st, out = gpu_ssb(d_idx, d_off, wl, normalize=1, g_mode=g_mode, c=wl.aberr)
        ref = oracle_ssb(idx, off, wl, normalize=True, c=wl.aberr)
        assert out["status"] == 0
        assert rel_l2(out["T"], ref["T"]) <= TOL
        assert rel_l2(out["phi"], ref["phi"]) <= TOL
        # element by element, relative to each Q's own size (the division by the pair count)
        assert np.max(np.abs(out["T"] - ref["T"])) <= 1e-5 * np.max(np.abs(ref["T"]))
        # a second FINALIZE (the per-Q counts are rebuilt, G recomputed or from the stored values)
        phase = torch.zeros(wl.n_frames, dtype=torch.float32, device="cuda")
        st.finalize(c=wl.aberr, phase=phase)
        assert rel_l2(phase.cpu().numpy().reshape(wl.scan), ref["phi"]) <= TOL


@pytest.mark.parametrize("name", ["small", "mid", "rect", "aberr", "n512", "n1024", "wide"])
def test_pair_count_matches_oracle(gpu, name):
    """The state's first counter is the number of (pixel, Q) pairs in the double-overlap sets (the
    oracle's per-Q pair counts summed), however the sum ran: fused (interval table from the binning,
    or from the table kernel with aberrations or the global bin table), from a stored G (REFOCUS),
    or normalised per Q."""
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    H, W = wl.det
    ny, nx = wl.scan
    kc, _ = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    _, npair = ossb.ssb_sum(np.zeros((len(kc), ny, nx)), kc, wl.step, wl.dk, wl.lam, wl.r_bf)
    P = int(npair.sum())
    st, out = gpu_ssb(d_idx, d_off, wl, c=wl.aberr, g_mode=stem.STEM_G_STORE)
    s = st.stats()
    assert out["status"] == 0
    assert s[0] == P and s[1] >= 1 and s[2] > 0 and s[3] == 1
    st.refocus(c=wl.aberr)
    torch.cuda.synchronize()
    s = st.stats()
    assert s[0] == P and 0 < s[2] <= 8 * P  # the refocus reads stored pairs only
    # the refocus sum's pieces: at least one per column with pairs, at most the waves the GPU holds
    assert (npair.sum(axis=0) > 0).sum() <= s[1] <= max(256 * 20, nx)
    # the adjoint leaves the counters of the last sum
    phase = torch.zeros(wl.n_frames, dtype=torch.float32, device="cuda")
    st.refocus(c=wl.aberr, phase=phase)
    st.backward((-(2.0 / phase.numel()) * (phase - phase.mean())).contiguous(), c=wl.aberr)
    torch.cuda.synchronize()
    assert st.stats()[0] == P
    # per Q: the normalised sum's pair counts equal the oracle's, frequency by frequency
    stn, outn = gpu_ssb(d_idx, d_off, wl, c=wl.aberr, normalize=1)
    assert outn["status"] == 0 and stn.stats()[0] == P
    assert np.array_equal(state_npair(stn, wl), npair)
    # G recomputed in several chunks of pixels: the same count
    str_, outr = gpu_ssb(d_idx, d_off, wl, c=wl.aberr, g_mode=stem.STEM_G_RECOMPUTE, scratch_mib=1)
    assert outr["status"] == 0 and str_.stats()[0] == P


def test_refocus_matches_fresh_reconstruction(gpu):
    """Interactive refocus (Sec. IV): only Eq. 3 and the phase are recomputed from stored G."""
    wl, idx, off = data("aberr")
    d_idx, d_off = to_device(idx, off)
    st, out0 = gpu_ssb(d_idx, d_off, wl, c=(0.0,) * 8)
    F = wl.n_frames
    phase = torch.zeros(F, dtype=torch.float32, device="cuda")
    T = torch.zeros(F, dtype=torch.complex64, device="cuda")
    st.refocus(c=wl.aberr, phase=phase, T=T)
    ref = oracle_ssb(idx, off, wl, c=wl.aberr)
    assert rel_l2(T.cpu().numpy().reshape(wl.scan), ref["T"]) <= TOL
    assert rel_l2(phase.cpu().numpy().reshape(wl.scan), ref["phi"]) <= TOL


@pytest.mark.parametrize("scratch_mib", [0, 1])
@pytest.mark.parametrize("name", ["small", "mid", "aberr"])
def test_recompute_mode_matches_oracle(gpu, name, scratch_mib):
    """G-recompute mode: the state keeps the binned counts only; every sum transforms chunks of
    pixels in a bounded scratch (1 MiB: several chunks), so a second FINALIZE with other
    coefficients works, and the adjoint recomputes G the same way."""
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    c = wl.aberr
    st, out = gpu_ssb(d_idx, d_off, wl, c=c, g_mode=stem.STEM_G_RECOMPUTE, scratch_mib=scratch_mib)
    if scratch_mib:
        assert st.stats()[3] > 1
    ref = oracle_ssb(idx, off, wl, c=c)
    assert out["status"] == 0
    assert rel_l2(out["T"], ref["T"]) <= TOL
    assert rel_l2(out["phi"], ref["phi"]) <= TOL
    assert st.pair_count() == int(sum(ossb.ssb_sum(ref["G"], ref["kc"], wl.step, wl.dk, wl.lam, wl.r_bf, c)[1].sum()
                                      for _ in [0]))
    # finalize again with different coefficients (the cube is intact)
    c2 = tuple(0.5 * v for v in C4_TRUE_ABERRATIONS)
    phase = torch.zeros(wl.n_frames, dtype=torch.float32, device="cuda")
    st.finalize(c=c2, phase=phase)
    ref2 = oracle_ssb(idx, off, wl, c=c2)
    assert rel_l2(phase.cpu().numpy().reshape(wl.scan), ref2["phi"]) <= TOL
    # adjoint with recomputed G
    phi = phase.view(-1)
    gbar = (-(2.0 / phi.numel()) * (phi - phi.mean())).contiguous()
    dc, dth = st.backward(gbar, c=c2)
    dco, dtho = ossb.ssb_adjoint(ref2["G"], ref2["kc"], ossb.neg_var_grad(ref2["phi"]), wl.step, wl.dk, wl.lam,
                                 wl.r_bf, c2)
    dc = dc.cpu().numpy()
    assert np.all(np.abs(dc - dco) <= 1e-4 * np.abs(dco) + 1e-6 * np.max(np.abs(dco)))
    assert rel_l2(dth.cpu().numpy(), dtho) <= 1e-4
    # REFOCUS in this mode runs the recomputed sum again
    st.refocus(c=c, phase=phase)
    assert rel_l2(phase.cpu().numpy().reshape(wl.scan), ref["phi"]) <= TOL


@pytest.mark.parametrize("prec", [stem.STEM_FFT_FP32, stem.STEM_DFT_BF16_SPLIT, stem.STEM_DFT_FP16_SPLIT],
                         ids=["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("name", ["small", "rect", "n512", "n1024"])
def test_zero_aberration_sum_equals_general_sum(gpu, name, prec):
    """With chi identically zero and no theta the fused sum adds G itself; given theta = 0 it takes
    the general path, whose phase factors are then exactly 1: the two agree bit for bit."""
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    det, _, optics = structs(wl)
    zeros = np.zeros(stem.ssb_num_pixels(det, optics), dtype=np.float32)
    _, fast = gpu_ssb(d_idx, d_off, wl, g_mode=stem.STEM_G_RECOMPUTE, precision=prec)
    _, gen = gpu_ssb(d_idx, d_off, wl, theta=zeros, g_mode=stem.STEM_G_RECOMPUTE, precision=prec)
    assert np.array_equal(fast["T"], gen["T"])
    assert np.array_equal(fast["phi"], gen["phi"])
    ref = oracle_ssb(idx, off, wl)
    assert rel_l2(fast["phi"], ref["phi"]) <= (TOL if prec == stem.STEM_FFT_FP32 else 1e-4)


def test_chunked_accumulate_equals_oneshot(gpu):
    wl, idx, off = data("mid")
    d_idx, d_off = to_device(idx, off)
    _, one = gpu_ssb(d_idx, d_off, wl)
    _, chk = gpu_ssb(d_idx, d_off, wl, chunk_rows=16)
    _, odd = gpu_ssb(d_idx, d_off, wl, chunk_rows=24)  # ragged last chunk
    assert rel_l2(chk["phi"], one["phi"]) <= 1e-6
    assert rel_l2(odd["phi"], one["phi"]) <= 1e-6


def test_uint16_cube_and_overflow(gpu):
    """A pile-up of 300 events in one bin does not fit uint8: STEM_EOVERFLOW, never clamped
    silently; the uint16 cube holds it and matches the oracle."""
    wl, idx, off = data("small")
    H, W = wl.det
    idx2, off2 = with_pileup(idx, off, 100, (H // 2) * W + W // 2, 300)
    d_idx, d_off = to_device(idx2, off2)
    st8, out8 = gpu_ssb(d_idx, d_off, wl, d_bits=8)
    assert out8["status"] & 8
    st16, out16 = gpu_ssb(d_idx, d_off, wl, d_bits=16)
    assert out16["status"] == 0
    ref = oracle_ssb(idx2, off2, wl)
    assert np.array_equal(state_D(st16, wl), ref["D"])
    assert rel_l2(out16["phi"], ref["phi"]) <= TOL


def test_ingest_copy_and_validation(gpu):
    """eer_load_csr: chunked host->device copy, then the device-side checks."""
    wl, idx, off = data("small")
    det, scan, optics = structs(wl)
    F = wl.n_frames
    d_idx = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
    d_off = torch.zeros(F + 1, dtype=torch.int64, device="cuda")
    st = stem.status_tensor()
    h_idx = torch.from_numpy(idx).pin_memory()
    h_off = torch.from_numpy(off).pin_memory()
    for f0 in range(0, F, 256):
        nf = min(256, F - f0)
        e0, e1 = int(off[f0]), int(off[f0 + nf])
        stem.eer_load_csr(h_idx[e0:e1], h_off[f0:f0 + nf + 1], f0, nf, e1 - e0, det, d_idx, d_off, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(d_idx.cpu().numpy(), idx) and np.array_equal(d_off.cpu().numpy(), off)
    # out-of-range index -> ERANGE (validate-only path)
    bad = idx.copy()
    bad[5] = W_H = wl.det[0] * wl.det[1]
    b_idx, b_off = to_device(bad, off)
    st.zero_()
    stem.eer_load_csr(None, None, 0, F, len(bad), det, b_idx, b_off, d_status=st)
    assert int(st.item()) == 2
    # decreasing offsets -> EOFFSETS
    off_bad = off.copy()
    off_bad[10] = off_bad[11] + 1
    b_idx, b_off = to_device(idx, off_bad)
    st.zero_()
    stem.eer_load_csr(None, None, 0, F, len(idx), det, b_idx, b_off, d_status=st)
    assert int(st.item()) & 4
    # offsets pointing past the event array -> EOFFSETS, never followed
    off_big = off.copy()
    off_big[-1] = len(idx) + 1000
    b_idx, b_off = to_device(idx, off_big)
    st.zero_()
    stem.eer_load_csr(None, None, 0, F, len(idx), det, b_idx, b_off, d_status=st)
    assert int(st.item()) & 4
    # COM and binning skip (and report) out-of-range indices without faulting
    b_idx, b_off = to_device(bad, off)
    g = gpu_com(b_idx, b_off, wl)
    assert g["status"] == 2
    assert W_H > 0


# ----------------------------------------------------------------------------------------------
# adjoint


def test_adjoint_matches_oracle_gradient(gpu):
    wl, idx, off = data("aberr")
    d_idx, d_off = to_device(idx, off)
    rng = np.random.default_rng(7)
    c = np.array(C4_TRUE_ABERRATIONS) * (1 + rng.uniform(-0.5, 0.5, size=8))
    st, out = gpu_ssb(d_idx, d_off, wl, c=c)
    phi = torch.from_numpy(out["phi"]).cuda()
    gbar = (-(2.0 / phi.numel()) * (phi - phi.mean())).contiguous().view(-1)
    dc, dth = st.backward(gbar, c=c)
    ref = oracle_ssb(idx, off, wl, c=c)
    gbar_o = ossb.neg_var_grad(ref["phi"])
    dco, dtho = ossb.ssb_adjoint(ref["G"], ref["kc"], gbar_o, wl.step, wl.dk, wl.lam, wl.r_bf, c)
    dc = dc.cpu().numpy()
    # every component, including those 1000x below the largest, to 1e-4 of its own size
    assert np.all(np.abs(dc - dco) <= 1e-4 * np.abs(dco) + 1e-7 * np.max(np.abs(dco)))
    assert rel_l2(dth.cpu().numpy(), dtho) <= 1e-4


def test_autograd_function_and_finite_differences(gpu):
    """SSBPhase: torch.autograd gradient of -Var(phi) equals central differences of the
    GPU forward (rel <= 1e-3) for the coefficients that carry at least 10% of the largest
    gradient.  (Smaller components sit below the FP32 forward's finite-difference noise;
    they are checked component by component against the FP64 oracle gradient above.)"""
    wl, idx, off = data("aberr")
    d_idx, d_off = to_device(idx, off)
    det, scan, optics = structs(wl)
    st = stem.SsbState(det, scan, optics)
    st.accumulate(d_idx, d_off, 0, wl.n_frames)
    rng = np.random.default_rng(8)
    c0 = np.array(C4_TRUE_ABERRATIONS) * (1 + rng.uniform(-0.5, 0.5, size=8))
    c = torch.tensor(c0, dtype=torch.float64, requires_grad=True)

    def loss_of(cc):
        phi = stem.SSBPhase.apply(cc, None, st)
        return -phi.double().var(unbiased=False)

    L = loss_of(c)
    L.backward()
    g = c.grad.numpy()
    for j in range(8):
        if abs(g[j]) < 0.1 * np.max(np.abs(g)):
            continue
        # fourth-order central differences with a step of 1% of the coefficient: the truncation
        # error (~1e-8 relative) stays far below the FP32 forward's rounding noise divided by h
        h = 1e-2 * abs(c0[j])
        vals = []
        for k in (-2, -1, 1, 2):
            ck = c0.copy()
            ck[j] += k * h
            with torch.no_grad():
                vals.append(float(loss_of(torch.tensor(ck)).double()))
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert abs(g[j] - fd) <= 1e-3 * abs(fd)
