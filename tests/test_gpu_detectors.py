"""Virtual detectors from events (Table 1 'radial sum' and 'sum all frames') against the oracle:
integer outputs, compared bit for bit."""
import numpy as np
import pytest
import torch

import paper_2104_06336_amd as stem
from gen import WORKLOADS, random_csr, simulate, with_pileup
from oracle import eer as oeer

from helpers import structs, to_device
from test_gpu_parity import data

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)


# bright field, an annulus across the disk edge, dark field, the whole detector, an empty one
ANNULI = ([0.0, 12.5, 17.0, 0.0, 5.0], [16.0, 20.0, 1e6, 1e6, 5.0])


@pytest.mark.parametrize("name", ["small", "mid", "rect"])
def test_virtual_annular_bit_exact(gpu, name):
    wl, idx, off = data(name)
    d_idx, d_off = to_device(idx, off)
    det, scan, _ = structs(wl)
    H, W = wl.det
    F = wl.n_frames
    r_in, r_out = ANNULI
    if name == "mid":  # 576 detector: scale the radii with the bright-field disk
        r_in, r_out = [v * wl.r_bf / 16 for v in r_in], [v * wl.r_bf / 16 for v in r_out]
    out = torch.full((len(r_in) * F,), -1, dtype=torch.int32, device="cuda")
    st = stem.status_tensor()
    stem.virtual_annular(d_idx, d_off, 0, F, det, scan, r_in, r_out, out, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = oeer.radial_sum(idx, off, W, H, r_in, r_out)
    assert np.array_equal(out.cpu().numpy().reshape(len(r_in), F), ref)
    assert np.array_equal(ref[3], oeer.frame_counts(off))


def test_virtual_annular_chunks_and_edge_frames(gpu):
    """Frame ranges that start and end inside a workgroup, empty frames, a pile-up, and the
    largest annulus count."""
    rng = np.random.default_rng(31)
    W, H = 40, 36
    idx, off = random_csr(rng, 3000, W, H, 25.0, p_empty=0.2)
    idx, off = with_pileup(idx, off, 1000, 18 * W + 20, 400)
    d_idx, d_off = to_device(idx, off)
    det = stem.Det(W, H, W // 2, H // 2, 1)
    scan = stem.Scan(50, 60, 0.2)
    F = 3000
    r_in = [0.5 * j for j in range(16)]
    r_out = [0.5 * j + 3.0 for j in range(16)]
    out = torch.full((16 * F,), -7, dtype=torch.int32, device="cuda")
    for f0, nf in ((0, 700), (700, 1), (701, 1299), (2000, 1000)):
        stem.virtual_annular(d_idx, d_off, f0, nf, det, scan, r_in, r_out, out)
    torch.cuda.synchronize()
    ref = oeer.radial_sum(idx, off, W, H, r_in, r_out)
    assert np.array_equal(out.cpu().numpy().reshape(16, F), ref)


def test_sum_frames_bit_exact_and_mean(gpu):
    wl, idx, off = data("mid")
    d_idx, d_off = to_device(idx, off)
    det, _, _ = structs(wl)
    H, W = wl.det
    F = wl.n_frames
    s = torch.zeros(W * H, dtype=torch.int32, device="cuda")
    mean = torch.zeros(W * H, dtype=torch.float32, device="cuda")
    st = stem.status_tensor()
    stem.sum_frames(d_idx, d_off, 0, F, det, s, mean, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = oeer.sum_frames(idx, off, W, H)
    got = s.cpu().numpy().view(np.uint32).reshape(H, W).astype(np.int64)
    assert np.array_equal(got, ref)
    assert np.array_equal(mean.cpu().numpy().reshape(H, W), (ref / F).astype(np.float32))
    # accumulated over chunks (a frame range that splits the event windows)
    s.zero_()
    for f0, nf in ((0, 1000), (1000, 1), (1001, F - 1001)):
        stem.sum_frames(d_idx, d_off, f0, nf, det, s)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy().view(np.uint32).reshape(H, W).astype(np.int64), ref)


def test_sum_frames_small_detector_and_range_errors(gpu):
    """A detector smaller than the LDS box, out-of-range indices (skipped and reported)."""
    rng = np.random.default_rng(32)
    W, H = 20, 12
    idx, off = random_csr(rng, 500, W, H, 30.0)
    bad = idx.copy()
    bad[17] = W * H + 3
    bad[400] = -1
    d_idx, d_off = to_device(bad, off)
    det = stem.Det(W, H, W // 2, H // 2, 1)
    s = torch.zeros(W * H, dtype=torch.int32, device="cuda")
    st = stem.status_tensor()
    stem.sum_frames(d_idx, d_off, 0, 500, det, s, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 2  # STEM_ERANGE
    keep = np.ones(len(bad), dtype=bool)
    keep[[17, 400]] = False
    ref = np.bincount(bad[keep].astype(np.int64), minlength=W * H).reshape(H, W)
    assert np.array_equal(s.cpu().numpy().reshape(H, W).astype(np.int64), ref)


def test_virtual_detectors_full_size(gpu):
    """scan1024 (4.2e7 events): bright-field / annular dark-field images and the PACBED pattern."""
    wl = WORKLOADS["scan1024"]
    d = simulate(wl, device="cuda")
    torch.cuda.synchronize()
    idx, off = d.idx.cpu().numpy(), d.off.cpu().numpy()
    det, scan, _ = structs(wl)
    H, W = wl.det
    F = wl.n_frames
    r_in, r_out = [0.0, 1.2 * wl.r_bf], [wl.r_bf, 4.0 * wl.r_bf]
    out = torch.zeros(2 * F, dtype=torch.int32, device="cuda")
    stem.virtual_annular(d.idx, d.off, 0, F, det, scan, r_in, r_out, out)
    s = torch.zeros(W * H, dtype=torch.int32, device="cuda")
    stem.sum_frames(d.idx, d.off, 0, F, det, s)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(2, F), oeer.radial_sum(idx, off, W, H, r_in, r_out))
    assert np.array_equal(s.cpu().numpy().reshape(H, W).astype(np.int64), oeer.sum_frames(idx, off, W, H))
