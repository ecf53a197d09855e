"""Run-length form -> linear indices on the GPU against the oracle's re-coding (integer, bit for
bit), and the reductions on the decoded events."""
import numpy as np
import pytest
import torch

import paper_2104_06336_amd as stem
from gen import WORKLOADS, random_csr, simulate
from oracle import eer as oeer

from helpers import structs, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)


def test_decode_rle_random_frames_and_chunks(gpu):
    rng = np.random.default_rng(51)
    W, H = 64, 48
    idx, off = random_csr(rng, 5000, W, H, 30.0, p_empty=0.15, sort=False)
    dist = oeer.rle_encode(idx, off).astype(np.int32)
    ref = oeer.rle_decode(dist, off)
    d_dist, d_off = to_device(dist, off)
    det = stem.Det(W, H, W // 2, H // 2, 1)
    out = torch.full((len(dist),), -5, dtype=torch.int32, device="cuda")
    st = stem.status_tensor()
    for f0, nf in ((0, 1), (1, 2000), (2001, 999), (3000, 2000)):
        stem.eer_decode_rle(d_dist, d_off, f0, nf, det, out, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out.cpu().numpy(), ref)


def test_decode_rle_out_of_range(gpu):
    """A negative distance or a sum past the detector: -1 and STEM_ERANGE, the rest intact."""
    W, H = 8, 8
    off = np.array([0, 3, 5, 8], dtype=np.int64)
    dist = np.array([3, 4, 60, 10, -20, 1, 1, 1], dtype=np.int32)
    d_dist, d_off = to_device(dist, off)
    out = torch.zeros(8, dtype=torch.int32, device="cuda")
    st = stem.status_tensor()
    stem.eer_decode_rle(d_dist, d_off, 0, 3, stem.Det(W, H, 4, 4, 1), out, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 2
    assert out.cpu().numpy().tolist() == [3, 7, -1, 10, -1, 1, 2, 3]


def test_decode_rle_full_size_then_reduce(gpu):
    """scan1024 (4.2e7 events) in run-length form: decoded indices equal the sorted events, and
    the centre of mass of the decoded events equals the oracle's."""
    wl = WORKLOADS["scan1024"]
    d = simulate(wl, device="cuda")
    torch.cuda.synchronize()
    idx, off = d.idx.cpu().numpy(), d.off.cpu().numpy()
    dist = oeer.rle_encode(idx, off).astype(np.int32)
    d_dist = torch.from_numpy(dist).cuda()
    out = torch.empty_like(d.idx)
    det, scan, optics = structs(wl)
    st = stem.status_tensor()
    stem.eer_decode_rle(d_dist, d.off, 0, wl.n_frames, det, out, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out.cpu().numpy(), oeer.rle_decode(dist, off))
    F = wl.n_frames
    com64 = torch.zeros(2 * F, dtype=torch.float64, device="cuda")
    stem.com_dpc(out, d.off, 0, F, det, scan, optics, None, com64=com64)
    H, W = wl.det
    cx, cy, *_ = oeer.com(idx, off, W, H)
    c = com64.cpu().numpy().reshape(2, F)
    assert np.array_equal(c[0], cx) and np.array_equal(c[1], cy)
