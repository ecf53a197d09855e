"""Degenerate and irregular inputs of the sideband path against the FP64 oracle.

- random hits over the whole detector (most outside the bright-field disk), 40% empty frames,
  unsorted frames, a 300-event pile-up on one kept pixel, on a 48 x 40 scan (other-length
  transforms) and a 32 x 64 scan (fused kernels), both G modes: D bit-exact, T and phi 1e-5;
- every event outside the kept bins: D = 0, T = 0 and phi = 0 exactly;
- a disk so small that one bin is kept (Kc = 0): the double-overlap set {|Q| < r, |Q| >= r} is
  empty, so T = 0 exactly and the pair count is 0;
- a single event in the whole scan;
- REFOCUS and the adjoint over the stored values on the irregular data (the balanced pieces of
  those sums over sparse and pile-up columns, other-length and fused scans), and on the
  degenerate cases (no kept events: T, phi and the gradients 0; no double-overlap pair: the same);
- REFOCUS and the adjoint on a state that no FINALIZE has marked: STEM_ESTATE, and after a
  FINALIZE both run clean, REFOCUS at FINALIZE's coefficients giving its phase; a later
  accumulation from frame 0 voids the FINALIZE again.
"""
import numpy as np
import pytest
import torch

import paper_2104_06336_amd as stem
from gen import WORKLOADS, random_csr, shuffle_within_frames, with_pileup
from oracle import eer as oeer
from oracle import ssb as ossb

from helpers import gpu_ssb, oracle_ssb, rel_l2, state_D, structs, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-5
SMALL = WORKLOADS["small"]
MODES = [stem.STEM_G_STORE, stem.STEM_G_RECOMPUTE]


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)


@pytest.mark.parametrize("g_mode", MODES, ids=["store", "recompute"])
@pytest.mark.parametrize("scan", [(48, 40), (32, 64)], ids=["48x40", "32x64"])
def test_random_hits_empty_frames_pileup(gpu, scan, g_mode):
    wl = SMALL.replace(scan=scan)
    H, W = wl.det
    rng = np.random.default_rng(21)
    idx, off = random_csr(rng, wl.n_frames, W, H, mean=30.0, p_empty=0.4, sort=False)
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    kept_pixel = int(np.flatnonzero(lut.reshape(-1) >= 0)[len(kc) // 2])
    idx, off = with_pileup(idx, off, 7, kept_pixel, 300)
    idx = shuffle_within_frames(rng, idx, off)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, c=(30.0, 5.0, -5.0, 0, 0, 0, 0, 0), g_mode=g_mode, d_bits=16)
    ref = oracle_ssb(idx, off, wl, c=(30.0, 5.0, -5.0, 0, 0, 0, 0, 0))
    assert out["status"] == 0
    assert np.array_equal(state_D(st, wl), ref["D"])
    assert rel_l2(out["T"], ref["T"]) <= TOL
    assert rel_l2(out["phi"], ref["phi"]) <= TOL


@pytest.mark.parametrize("g_mode", MODES, ids=["store", "recompute"])
def test_all_events_outside_the_kept_bins(gpu, g_mode):
    wl = SMALL.replace(scan=(32, 48))
    H, W = wl.det
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    outside = np.flatnonzero(lut.reshape(-1) < 0).astype(np.int32)
    rng = np.random.default_rng(5)
    n = rng.poisson(10.0, size=wl.n_frames)
    off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    idx = rng.choice(outside, size=int(off[-1])).astype(np.int32)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, g_mode=g_mode)
    assert out["status"] == 0
    assert not state_D(st, wl).any()
    assert not out["T"].any() and not out["phi"].any()


@pytest.mark.parametrize("g_mode", MODES, ids=["store", "recompute"])
def test_one_kept_bin_has_empty_sets(gpu, g_mode):
    wl = SMALL.replace(scan=(32, 32), r_bf=0.9)
    det, _, optics = structs(wl)
    assert stem.ssb_num_pixels(det, optics) == 1
    H, W = wl.det
    rng = np.random.default_rng(9)
    idx, off = random_csr(rng, wl.n_frames, W, H, mean=20.0)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, g_mode=g_mode)
    ref = oracle_ssb(idx, off, wl)
    assert out["status"] == 0
    assert np.array_equal(state_D(st, wl), ref["D"])
    assert not ref["T"].any()
    assert not out["T"].any() and not out["phi"].any()
    assert st.pair_count() == 0


@pytest.mark.parametrize("g_mode", MODES, ids=["store", "recompute"])
def test_single_event(gpu, g_mode):
    wl = SMALL.replace(scan=(32, 32))
    H, W = wl.det
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    pixel = int(np.flatnonzero(lut.reshape(-1) >= 0)[3])
    off = np.zeros(wl.n_frames + 1, dtype=np.int64)
    off[418:] = 1  # frame 417 holds the one event
    idx = np.array([pixel], dtype=np.int32)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, g_mode=g_mode)
    ref = oracle_ssb(idx, off, wl)
    assert out["status"] == 0
    assert np.array_equal(state_D(st, wl), ref["D"])
    assert rel_l2(out["T"], ref["T"]) <= TOL
    assert rel_l2(out["phi"], ref["phi"]) <= TOL


def _irregular(wl, seed=21):
    H, W = wl.det
    rng = np.random.default_rng(seed)
    idx, off = random_csr(rng, wl.n_frames, W, H, mean=30.0, p_empty=0.4, sort=False)
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    kept_pixel = int(np.flatnonzero(lut.reshape(-1) >= 0)[len(kc) // 2])
    idx, off = with_pileup(idx, off, 7, kept_pixel, 300)
    return idx, off


@pytest.mark.parametrize("scan", [(48, 40), (32, 64)], ids=["48x40", "32x64"])
def test_refocus_and_adjoint_on_irregular_data(gpu, scan):
    wl = SMALL.replace(scan=scan)
    idx, off = _irregular(wl)
    d_idx, d_off = to_device(idx, off)
    c1 = (30.0, 5.0, -5.0, 0, 0, 0, 0, 0)
    st, out = gpu_ssb(d_idx, d_off, wl, c=c1, g_mode=stem.STEM_G_STORE, d_bits=16)
    assert out["status"] == 0
    # refocus with other coefficients and a probe phase, against a fresh oracle reconstruction
    c2 = (-20.0, 2.0, 8.0, 150.0, -200.0, 100.0, 250.0, 5.0e3)
    theta = np.random.default_rng(3).uniform(-0.3, 0.3, size=st.n_k).astype(np.float32)
    phase = torch.zeros(wl.n_frames, dtype=torch.float32, device="cuda")
    T = torch.zeros(wl.n_frames, dtype=torch.complex64, device="cuda")
    st.refocus(c=c2, theta=torch.from_numpy(theta).cuda(), phase=phase, T=T)
    ref = oracle_ssb(idx, off, wl, c=c2, theta=theta.astype(np.float64))
    assert rel_l2(T.cpu().numpy().reshape(wl.scan), ref["T"]) <= TOL
    assert rel_l2(phase.cpu().numpy().reshape(wl.scan), ref["phi"]) <= TOL
    # the adjoint over the stored values at those coefficients, against the oracle's gradient
    gbar = (-(2.0 / phase.numel()) * (phase - phase.mean())).contiguous()
    dc, dth = st.backward(gbar, c=c2, theta=torch.from_numpy(theta).cuda())
    dco, dtho = ossb.ssb_adjoint(ref["G"], ref["kc"], ossb.neg_var_grad(ref["phi"]), wl.step, wl.dk, wl.lam,
                                 wl.r_bf, c2, theta.astype(np.float64))
    assert rel_l2(dc.cpu().numpy(), dco) <= 1e-4
    assert rel_l2(dth.cpu().numpy(), dtho) <= 1e-4


def _zero_refocus_and_adjoint(st, wl):
    phase = torch.full((wl.n_frames,), 1.0, dtype=torch.float32, device="cuda")
    T = torch.full((wl.n_frames,), 1.0, dtype=torch.complex64, device="cuda")
    st.refocus(c=(10.0, 1.0, -1.0, 0, 0, 0, 0, 0), phase=phase, T=T)
    assert not T.any() and not phase.any()
    gbar = torch.linspace(-1.0, 1.0, wl.n_frames, dtype=torch.float32, device="cuda")
    dc, dth = st.backward(gbar, c=(10.0, 1.0, -1.0, 0, 0, 0, 0, 0))
    assert not dc.any() and not dth.any()


def test_refocus_and_adjoint_without_kept_events(gpu):
    wl = SMALL.replace(scan=(32, 48))
    H, W = wl.det
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    outside = np.flatnonzero(lut.reshape(-1) < 0).astype(np.int32)
    rng = np.random.default_rng(5)
    n = rng.poisson(10.0, size=wl.n_frames)
    off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    idx = rng.choice(outside, size=int(off[-1])).astype(np.int32)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, g_mode=stem.STEM_G_STORE)
    assert out["status"] == 0 and st.pair_count() > 0
    _zero_refocus_and_adjoint(st, wl)


def test_refocus_and_adjoint_without_pairs(gpu):
    wl = SMALL.replace(scan=(32, 32), r_bf=0.9)
    H, W = wl.det
    rng = np.random.default_rng(9)
    idx, off = random_csr(rng, wl.n_frames, W, H, mean=20.0)
    d_idx, d_off = to_device(idx, off)
    st, out = gpu_ssb(d_idx, d_off, wl, g_mode=stem.STEM_G_STORE)
    assert out["status"] == 0 and st.pair_count() == 0
    _zero_refocus_and_adjoint(st, wl)


@pytest.mark.parametrize("g_mode", MODES, ids=["store", "recompute"])
@pytest.mark.parametrize("scan", [(48, 40), (32, 64)], ids=["48x40", "32x64"])
def test_refocus_and_adjoint_need_a_finalize(gpu, scan, g_mode):
    wl = SMALL.replace(scan=scan)
    H, W = wl.det
    F = wl.n_frames
    idx, off = random_csr(np.random.default_rng(13), F, W, H, mean=30.0)
    d_idx, d_off = to_device(idx, off)
    det, scn, optics = structs(wl)
    st = stem.SsbState(det, scn, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, g_mode, 8), device="cuda")
    st.state.zero_()  # a fresh state: no FINALIZE mark
    st.accumulate(d_idx, d_off, 0, F)
    torch.cuda.synchronize()
    assert int(st.status.item()) == 0
    c = (10.0, 1.0, -1.0, 0, 0, 0, 0, 0)
    gbar = torch.linspace(-1.0, 1.0, F, dtype=torch.float32, device="cuda")
    phase = torch.zeros(F, dtype=torch.float32, device="cuda")
    st.refocus(c=c, phase=phase)
    torch.cuda.synchronize()
    assert int(st.status.item()) == stem.STEM_ESTATE
    st.status.zero_()
    st.backward(gbar, c=c)
    torch.cuda.synchronize()
    assert int(st.status.item()) == stem.STEM_ESTATE
    st.status.zero_()
    ref = torch.zeros(F, dtype=torch.float32, device="cuda")
    st.finalize(c=c, phase=ref)
    st.refocus(c=c, phase=phase)
    st.backward(gbar, c=c)
    torch.cuda.synchronize()
    assert int(st.status.item()) == 0
    assert rel_l2(phase.cpu().numpy(), ref.cpu().numpy()) <= TOL
    # a new accumulation from frame 0 voids that FINALIZE
    st.accumulate(d_idx, d_off, 0, F)
    st.refocus(c=c, phase=phase)
    torch.cuda.synchronize()
    assert int(st.status.item()) == stem.STEM_ESTATE
