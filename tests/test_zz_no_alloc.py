"""The allocation-free centre-of-mass + DPC entry point (com_dpc_noalloc) through the C ABI:
identical outputs to com_dpc with a caller workspace, on two calls in a row (the second on a
smaller scan), and its size limit."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2104_06336_amd as stem
from gen import random_csr

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _outputs(F, dev):
    return (torch.full((2 * F,), -1.0, dtype=torch.float64, device=dev),
            torch.full((2 * F,), -1.0, dtype=torch.float32, device=dev),
            torch.full((F,), -1, dtype=torch.int32, device=dev),
            torch.full((F,), -1.0, dtype=torch.float32, device=dev),
            torch.zeros(1, dtype=torch.int32, device=dev))


def _case(seed, ny, nx, W, H, dev):
    rng = np.random.default_rng(seed)
    idx, off = random_csr(rng, ny * nx, W, H, mean=12.0)
    d_idx = torch.from_numpy(idx).to(dev)
    d_off = torch.from_numpy(off).to(dev)
    det = stem.Det(W, H, W // 2, H // 2, 1)
    scan = stem.Scan(ny, nx, 0.2)
    optics = stem.Optics.from_values(0.0196875, 16.0, 0.0794)
    dpc = stem.Dpc(0.5, 0.01, 0.001, 12)
    return d_idx, d_off, det, scan, optics, dpc


def test_noalloc_matches_workspace_call_twice(gpu):
    lib = stem.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for seed, (ny, nx) in ((11, (256, 128)), (12, (32, 64))):  # second call: a smaller scan
        print(f"[no_alloc] seed {seed} scan {ny}x{nx}", flush=True)
        d_idx, d_off, det, scan, optics, dpc = _case(seed, ny, nx, 48, 40, gpu)
        F = ny * nx
        ref = _outputs(F, gpu)
        ws = torch.empty(stem.com_dpc_workspace_bytes(scan), dtype=torch.uint8, device=gpu)
        rc = lib.com_dpc(_p(d_idx), _p(d_off), 0, F, ctypes.byref(det), ctypes.byref(scan), ctypes.byref(optics),
                         ctypes.byref(dpc), _p(ref[0]), _p(ref[1]), _p(ref[2]), _p(ref[3]), _p(ws), ws.numel(),
                         _p(ref[4]), stream)
        assert rc == 0
        out = _outputs(F, gpu)
        rc = lib.com_dpc_noalloc(_p(d_idx), _p(d_off), 0, F, ctypes.byref(det), ctypes.byref(scan),
                                 ctypes.byref(optics), ctypes.byref(dpc), _p(out[0]), _p(out[1]), _p(out[2]),
                                 _p(out[3]), _p(out[4]), stream)
        assert rc == 0
        torch.cuda.synchronize()
        assert int(ref[4].item()) == 0 and int(out[4].item()) == 0
        for a, b in zip(ref[:4], out[:4]):
            assert torch.equal(a, b)
        assert float(out[3].abs().max()) > 0


def test_noalloc_rejects_scans_beyond_its_workspace(gpu):
    lib = stem.lib()
    assert lib.com_dpc_noalloc_max_workspace() == 16 << 20
    d_idx, d_off, det, _, optics, dpc = _case(13, 32, 32, 48, 40, gpu)
    big = stem.Scan(2048, 1024, 0.2)  # 3 half-spectrum planes of 25 MB each
    assert stem.com_dpc_workspace_bytes(big) > lib.com_dpc_noalloc_max_workspace()
    F = 2048 * 1024
    com = torch.zeros(2 * F, dtype=torch.float64, device=gpu)
    ph = torch.zeros(F, dtype=torch.float32, device=gpu)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.com_dpc_noalloc(_p(d_idx), _p(d_off), 0, 0, ctypes.byref(det), ctypes.byref(big), ctypes.byref(optics),
                             ctypes.byref(dpc), _p(com), None, None, _p(ph), None, stream)
    assert rc == 16  # STEM_EWORKSPACE
