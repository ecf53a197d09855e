#!/usr/bin/env python
"""Throughput of the event-based phase-contrast path on one MI355X.

One step = the whole hot path over one synthetic acquisition already resident in HBM:
centre of mass of every frame + DPC integration (com_dpc), then the single-sideband
reconstruction (ssb_reconstruct, one shot: binning, scan transform, double-overlap sum,
phase image).  Reported: events/s (value) and scan positions/s, per-step median and minimum,
the per-kernel roofline of the dominant kernel, the split-precision scan-DFT variants with their
error against the FP64 oracle, and the oracle itself timed on the host (1 thread and all cores).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload scan1024]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/s + scan positions/s, COM-DPC+SSB; BF16-split vs FP32 at <=1e-4 error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CPU_WORKERS_MAX = 16   # the host cores one GPU's share of a box provides


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------------
# bytes each kernel must move (the measurement plan's per-position figures, per kernel)

def algorithmic_bytes(name, g):
    """(bytes per step by the measurement plan, bytes per step including the binned cube's round
    trip) of the kernels named name, or None.

    The plan counts, per scan position: events 4N + 8 for each pass over them, COM out, the
    row-transformed half spectrum X written once and read once (16 n_K (Nx/2+1)/Nx), the stored
    double-overlap values (8 per pair each way), and 28 bytes for T, the inverse FFT round trip and
    phi.  The uint8 binned cube D between binning and row transform is not in the plan (it assumed
    the two fused); its bytes are the second figure.  The fused sum is billed for the columns it
    actually reads (g["sum_read"], counted by the kernels), not the whole X.
    g: C (events), F (frames), nk, nx, ny, P (pairs), d_bytes, sum_read, store (1 when the
    stored-G FINALIZE writes the double-overlap values)."""
    C, F, nk, nx, ny = g["C"], g["F"], g["nk"], g["nx"], g["ny"]
    nh = nx // 2 + 1
    X = nk * nh * ny * 8
    Db = nk * F * g["d_bytes"]
    ev = 4 * C + 8 * (F + 1)
    pw = 8 * g["P"] if g.get("store") else 0
    table = {
        "com_moments": (ev + 16 * F, ev + 16 * F),
        "bin_densify": (ev, ev + Db),
        "bin_com": (ev + 16 * F, ev + 16 * F + Db),
        "xstage_fft": (X, X + Db),
        "xstage_mfma": (X, X + Db),
        "ssb_yreduce": (g["sum_read"] + pw, g["sum_read"] + pw),
        "ssb_yreduce_mfma": (g["sum_read"] + pw, g["sum_read"] + pw),
        "phase_fft": (28 * F, 28 * F),
        "dpc_rows": (16 * F + 16 * nh * ny, 16 * F + 16 * nh * ny),
        "dpc_cols": (24 * nh * ny, 24 * nh * ny),
        "dpc_fft": (8 * nh * ny + 4 * F, 8 * nh * ny + 4 * F),
    }
    return table.get(name)


def step_bytes(g):
    """Bytes of one whole step by the measurement plan: COM-DPC 4N + 8 + 8 + 44 and SSB
    4N + 8 + 16 n_K (Nx/2+1)/Nx + 28 per scan position (+ 8 per pair when the stored-G FINALIZE
    writes the double-overlap values)."""
    C, F, nk, nx, ny = g["C"], g["F"], g["nk"], g["nx"], g["ny"]
    return (4 * C + 60 * F) + (4 * C + 8 * F + 16 * nk * (nx // 2 + 1) * ny + 28 * F) + (8 * g["P"] if g.get("store") else 0)


def source_sha():
    h = hashlib.sha256()
    for d in ("paper_2104_06336_amd/csrc", "include"):
        for f in sorted(os.listdir(os.path.join(ROOT, d))):
            with open(os.path.join(ROOT, d, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM traffic per launch measured with rocprofv3 counters, if taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(f"{kernel}@{workload}")
    if not ent or ent.get("source_sha") != source_sha():
        return None
    return ent.get("bytes_per_launch")


# rocprofv3 kernel names of the kernels bench.py reports, by their trace name
PROFILED = {
    "stem::k_com": "com_moments",
    "stem::k_bin<unsigned char, true, false>": "bin_densify",
    "stem::k_xstage<stem::XfFft<1024>, unsigned char>": "xstage_fft",
    "stem::k_yreduce<stem::XfFft<1024>, true, false>": "ssb_yreduce",
    "stem::k_psum_stream<false>": "ssb_reduce",
    "stem::k_padj_stream": "ssb_adjoint_pruned",
    "stem::k_yadjoint<stem::XfFft<512> >": "ssb_yadjoint",
    "stem::k_dpc_cols<1024, 4>": "dpc_cols",
}


# kernels the benchmark runs on another workload than the timed step's (the adjoint extra)
PROFILED_WORKLOAD = {"ssb_adjoint_pruned": "aberrated512", "ssb_yadjoint": "aberrated512"}


def _pmc_rows(path):
    """Per-dispatch counter sums of a rocprofv3 --pmc CSV: {(dispatch, kernel, grid): {counter: value}}."""
    import csv
    rows = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]))
            rows.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return rows


def summarize_profile(d, workload):
    """Turns the CSVs of the three counter runs and the kernel-trace run (written by the
    commands in the profile notes) into profiles/traffic.json and markdown tables.

    Reads: raw TCC_EA0_RDREQ_{32B,64B,128B} request counts times their sizes, divided by the factor
    the same counters give for k_validate (a plain streaming read of 4C + 8(F+1) bytes; C and F
    from the JSON line of that run).  Writes: WRITE_SIZE (KiB) divided by its factor for the
    1 GiB device copy (the copy kernel whose grid covers 2^28 floats in 8-float pieces)."""
    out_line = [ln for ln in open(os.path.join(d, "RDREQ.out")) if ln.startswith("{")][-1]
    cfg = json.loads(out_line)["config"]
    C, F = cfg["events"], cfg["frames"]
    rd, wr = _pmc_rows(os.path.join(d, "RDREQ.csv")), _pmc_rows(os.path.join(d, "WRITE_SIZE.csv"))
    fetch = _pmc_rows(os.path.join(d, "FETCH_SIZE.csv")) if os.path.exists(os.path.join(d, "FETCH_SIZE.csv")) else {}

    def rbytes(c):
        return (32 * c.get("TCC_EA0_RDREQ_32B_sum", 0) + 64 * c.get("TCC_EA0_RDREQ_64B_sum", 0)
                + 128 * c.get("TCC_EA0_RDREQ_128B_sum", 0))

    def per_kernel(rows, name, f):
        v = [f(c) for (_, k, _), c in rows.items() if k.startswith(("void " + name + "(", name + "("))]
        return (statistics.mean(v), len(v)) if v else (None, 0)

    # the ingest of the whole event list (the largest k_validate dispatch; a streamed ingest
    # validates chunks)
    val = max(rbytes(c) for (_, k, _), c in rd.items() if k.startswith("stem::k_validate("))
    read_factor = val / (4 * C + 8 * (F + 1))
    copies = [c["WRITE_SIZE"] * 1024 for (_, k, g), c in wr.items() if "direct_copy" in k and g == 33546240]
    write_factor = statistics.mean(copies) / (1 << 30)
    sha = source_sha()
    rec = {}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(path):
        # entries of other runs on the same sources are kept
        with open(path) as fh:
            rec = {k: v for k, v in json.load(fh).items() if isinstance(v, dict) and v.get("source_sha") == sha}
    rec.update({"_note": summarize_profile.__doc__.split("\n\n")[1].replace("\n    ", " ").strip(),
                "read_factor": round(read_factor, 5), "write_factor": round(write_factor, 5)})
    lines = ["| Kernel | Trace name | Dispatches | FETCH_SIZE (MB, raw) | Reads (MB, calibrated) "
             "| Writes (MB, calibrated) |", "|---|---|---:|---:|---:|---:|"]
    for kname, tname in PROFILED.items():
        r, n = per_kernel(rd, kname, rbytes)
        w, _ = per_kernel(wr, kname, lambda c: c["WRITE_SIZE"] * 1024)
        fs, _ = per_kernel(fetch, kname, lambda c: c["FETCH_SIZE"] * 1024)
        if r is None or w is None:
            continue
        r, w = r / read_factor, w / write_factor
        wl_k = PROFILED_WORKLOAD.get(tname, workload)
        rec[f"{tname}@{wl_k}"] = {"bytes_per_launch": int(r + w), "read_bytes": int(r), "write_bytes": int(w),
                                  "source_sha": sha}
        lines.append(f"| `{kname}` | {tname}@{wl_k} | {n} | {fs / 1e6 if fs else float('nan'):.1f} | {r / 1e6:.1f} "
                     f"| {w / 1e6:.1f} |")
    rec = {k: rec[k] for k in ["_note", "read_factor", "write_factor"] + sorted(k for k in rec if "@" in k)}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(f"C = {C}, F = {F}; read factor {read_factor:.5f} (k_validate), write factor {write_factor:.5f} "
          f"(1 GiB copy, {len(copies)} dispatches); sources sha {sha}\n")
    print("\n".join(lines))
    sq_path = os.path.join(d, "SQ.csv")
    if os.path.exists(sq_path):
        # instruction and wave counters: per launch means, and the derived VALU busy fraction
        # (SQ_ACTIVE_INST_VALU cycles x 4 / (GRBM_GUI_ACTIVE x the 256 x 4 SIMDs / 8 XCDs))
        sq = _pmc_rows(sq_path)
        names = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_ACTIVE_INST_VALU",
                 "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"]
        print("\n| Kernel | " + " | ".join(names) + " | VALU busy | mean waves per CU |\n|---|"
              + "---:|" * (len(names) + 2))
        for kname, tname in PROFILED.items():
            vals = {}
            for c in names:
                v, _ = per_kernel(sq, kname, lambda r, c=c: r.get(c, float("nan")))
                vals[c] = v
            if vals["SQ_WAVES"] is None:
                continue
            busy = vals["GRBM_GUI_ACTIVE"] / 8 if vals["GRBM_GUI_ACTIVE"] else float("nan")
            valu = vals["SQ_ACTIVE_INST_VALU"] * 4 / (busy * 1024) if busy == busy and busy > 0 else float("nan")
            occ = vals["SQ_WAVE_CYCLES"] / (busy * 256) if busy == busy and busy > 0 else float("nan")
            print(f"| `{kname}` | " + " | ".join(f"{vals[c]:.4g}" for c in names) + f" | {valu:.3f} | {occ:.1f} |")
    stats = os.path.join(d, "kernel_stats.csv")
    if os.path.exists(stats):
        import csv
        print("\n| Kernel | Calls | Average µs | Min µs | Max µs |\n|---|---:|---:|---:|---:|")
        with open(stats, newline="") as fh:
            for r in csv.DictReader(fh):
                name = r["Name"].removeprefix("void ")
                if name.startswith("stem::"):
                    name = name[:name.rfind("(")] if name.endswith(")") else name
                    print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} "
                          f"| {float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")


# ----------------------------------------------------------------------------------------------
# the FP64 oracle on the host (the CPU baseline), 1 thread and all cores

def _oracle_frames(job):
    """One shard of frames: centre of mass and binned counts (oracle functions, this process)."""
    from oracle import eer as oeer
    idx, off, W, H, b, lut = job
    cx, cy, *_ = oeer.com(idx, off, W, H)
    return cx, cy, oeer.bin_counts(idx, off, W, b, lut).astype("uint16")


def _oracle_pixels(job):
    """One shard of kept pixels: their scan transform and their part of the Eq. 3 sum."""
    from oracle import ssb as ossb
    D, kc, ny, nx, step, dk, lam, r_bf, c = job
    G = ossb.scan_dft(ossb.cube(D, ny, nx))
    return ossb.ssb_sum(G, kc, step, dk, lam, r_bf, c)[0]


def oracle_single(idx, off, wl):
    """The oracle over the whole workload in this process (numpy runs these single-threaded),
    stage by stage; returns (seconds, stage seconds, reference outputs)."""
    from oracle import dpc as odpc
    from oracle import eer as oeer
    from oracle import ssb as ossb

    H, W = wl.det
    ny, nx = wl.scan
    t = {}
    t0 = time.perf_counter()
    cx, cy, *_ = oeer.com(idx, off, W, H)
    t["com"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    odpc.com_dpc(cx.reshape(ny, nx), cy.reshape(ny, nx), wl.dk, wl.step)
    t["dpc"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    D = oeer.bin_counts(idx, off, W, wl.bin, lut)
    t["bin"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    G = ossb.scan_dft(ossb.cube(D, ny, nx))
    t["scan_dft"] = time.perf_counter() - t0
    del D
    t0 = time.perf_counter()
    T, npair = ossb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf, wl.aberr)
    t["ssb_sum"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    phi = ossb.phase_from_T(T)
    t["phase"] = time.perf_counter() - t0
    return sum(t.values()), t, {"kc": kc, "G": G, "T": T, "phi": phi, "npair": npair}


def oracle_parallel(pool, n_workers, idx, off, wl):
    """The same oracle functions over frame shards (COM, binning) and pixel shards (scan transform
    and Eq. 3 sum) in n_workers processes; DPC and the phase transform in this one."""
    import numpy as np

    from oracle import dpc as odpc
    from oracle import eer as oeer
    from oracle import ssb as ossb

    H, W = wl.det
    ny, nx = wl.scan
    F = wl.n_frames
    t = {}
    t0 = time.perf_counter()
    kc, lut = oeer.bin_geometry(W, H, wl.bin, wl.r_bf)
    rows = np.linspace(0, ny, n_workers + 1).astype(int)
    jobs = []
    for a, b in zip(rows[:-1], rows[1:]):
        f0, f1 = a * nx, b * nx
        e0, e1 = int(off[f0]), int(off[f1])
        jobs.append((idx[e0:e1], off[f0:f1 + 1] - e0, W, H, wl.bin, lut))
    parts = pool.map(_oracle_frames, jobs)
    cx = np.concatenate([p[0] for p in parts])
    cy = np.concatenate([p[1] for p in parts])
    D = np.concatenate([p[2] for p in parts], axis=1)
    t["com_bin"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    odpc.com_dpc(cx.reshape(ny, nx), cy.reshape(ny, nx), wl.dk, wl.step)
    t["dpc"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    pix = np.linspace(0, len(kc), n_workers + 1).astype(int)
    jobs = [(D[a:b], kc[a:b], ny, nx, wl.step, wl.dk, wl.lam, wl.r_bf, wl.aberr) for a, b in zip(pix[:-1], pix[1:])]
    T = sum(pool.map(_oracle_pixels, jobs))
    t["scan_dft_ssb_sum"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    phi = ossb.phase_from_T(T)
    t["phase"] = time.perf_counter() - t0
    return sum(t.values()), t, phi


def oracle_pruned_values(G, kc, wl):
    """The oracle's G on the double-overlap pairs in the library's stored order (scan-frequency
    column, then pixel, then ascending signed row frequency), for the error of the stored G."""
    import numpy as np

    from oracle import ssb as ossb
    ny, nx = wl.scan
    qx, qy = ossb.scan_q_grid(ny, nx, wl.step, wl.dk)
    order = np.argsort(ossb.signed_freq_index(ny), kind="stable")
    r2 = float(wl.r_bf) ** 2
    masks = [ossb.double_overlap(float(kc[kd, 0]), float(kc[kd, 1]), qx, qy, r2)[order].T for kd in range(len(kc))]
    sizes = np.stack([m.sum(axis=1) for m in masks], axis=1)  # [mx][kd]
    starts = (np.cumsum(sizes.ravel()) - sizes.ravel()).reshape(sizes.shape)
    out = np.empty(int(sizes.sum()), dtype=np.complex128)
    for kd, m in enumerate(masks):
        v = G[kd][order].T[m]  # pixel kd's values, column by column
        s = sizes[:, kd]
        out[np.repeat(starts[:, kd] - (np.cumsum(s) - s), s) + np.arange(len(v))] = v
    return out


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ----------------------------------------------------------------------------------------------


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scan1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision scan-DFT variants")
    ap.add_argument("--no-extras", action="store_true", help="skip the refocus, adjoint, detector and streaming timings")
    ap.add_argument("--g-mode", choices=("auto", "recompute", "store"), default="auto",
                    help="G mode of the timed step (auto: both are timed, the faster is the headline)")
    ap.add_argument("--scratch-mib", type=int, default=2048,
                    help="recompute scratch of the timed steps (2048: every pixel of scan1024 in one chunk; "
                         "the library's default, 64 MiB, is timed beside it)")
    ap.add_argument("--com-beside", choices=("finalize", "binning"), default="finalize",
                    help="where COM runs on the second stream: beside FINALIZE (with DPC), or from the start "
                         "of the step beside the binning (DPC still beside FINALIZE)")
    ap.add_argument("--fused-com", action="store_true",
                    help="centre of mass formed by the binning pass (ssb_reconstruct_com) instead of its own "
                         "pass over the events on the second stream")
    ap.add_argument("--schedules", choices=("both", "serial", "overlapped"), default="both",
                    help="step schedules timed (serial: one stream only, so that a kernel trace of the run "
                         "holds only dispatches that no other kernel shares the GPU with)")
    ap.add_argument("--no-default-scratch", action="store_true",
                    help="skip the step timed with the library's default recompute scratch (profiling runs)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run a device copy of this many MiB first (counter calibration)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="no GPU work: turn the rocprofv3 CSVs in DIR into profiles/traffic.json and tables")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.workload)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU mode "
              "(see the sharding notes in the design document); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline's worker processes start before anything touches the GPU
    pool, n_workers = None, 0
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        n_workers = max(1, min(CPU_WORKERS_MAX, os.cpu_count() or 1))
        pool = mp.get_context("fork").Pool(n_workers)

    import numpy as np
    import torch

    import paper_2104_06336_amd as stem
    from gen import C4_TRUE_ABERRATIONS, WORKLOADS, simulate

    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    H, W = wl.det
    ny, nx = wl.scan
    F = wl.n_frames

    t0 = time.time()
    data = simulate(wl, device=dev)
    torch.cuda.synchronize()
    d_idx, d_off = data.idx.contiguous(), data.off.contiguous()
    C = int(d_idx.numel())
    log(f"generated {args.workload}: {F} frames, {C} events in {time.time() - t0:.1f} s")

    det = stem.Det(W, H, W // 2, H // 2, wl.bin)
    scan = stem.Scan(ny, nx, wl.step)
    optics = stem.Optics.from_values(wl.lam, wl.r_bf, wl.dk, wl.aberr)
    dpc = stem.Dpc(0.5, 0.0, 0.0, 10)
    status = stem.status_tensor(dev)
    stem.eer_load_csr(None, None, 0, F, C, det, d_idx, d_off, d_status=status)
    stem.check_status(status, "event validation")

    com64 = torch.empty(2 * F, dtype=torch.float64, device=dev)
    phase_dpc = torch.empty(F, dtype=torch.float32, device=dev)
    ws = torch.empty(stem.com_dpc_workspace_bytes(scan), dtype=torch.uint8, device=dev)
    phase_ssb = torch.empty(F, dtype=torch.float32, device=dev)
    T_ssb = torch.empty(F, dtype=torch.complex64, device=dev)

    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    side = torch.cuda.Stream(device=dev)  # default priority
    main_stream = torch.cuda.current_stream(dev)
    G_MODES = {"recompute": stem.STEM_G_RECOMPUTE, "store": stem.STEM_G_STORE}

    def run(precision, g_mode, steps, warmup, overlap=True, opt=optics, trace=False, keep=False, scratch_mib=None):
        """Times `steps` whole steps; returns a dict with the elapsed seconds, the per-step times
        (HIP events between steps on the main stream), the kernel trace, the state's counters and,
        with keep, the SSB phase, T and the state.  With overlap, COM + DPC run on a second stream
        beside FINALIZE (after ACCUMULATE over all frames, the work of ONESHOT; the two share only
        the read-only events).  With trace, a HIP event pair brackets every kernel (per-kernel
        times); those records add queue packets between kernels, so step times come from runs
        without them."""
        mib = args.scratch_mib if scratch_mib is None else scratch_mib
        st = stem.SsbState(det, scan, opt, stem.Ssb(precision, 0, g_mode, 8, mib), device=dev)
        fused = args.fused_com
        com_kw = {"com64": com64} if fused else {}
        n_com = 0 if fused else F
        early_com = args.com_beside == "binning" and not fused

        def step():
            if overlap and early_com:
                side.wait_stream(main_stream)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, F, det, scan, com64=com64, d_status=status)
                st.accumulate(d_idx, d_off, 0, F)
                side.wait_stream(main_stream)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, 0, det, scan, optics, dpc, com64=com64, phase=phase_dpc,
                                 ws=ws, d_status=status)
                st.finalize(phase=phase_ssb, T=T_ssb)
                main_stream.wait_stream(side)
            elif overlap:
                # binning (+ COM) and, with stored G, the row transform first; DPC (latency-bound) then
                # runs beside the column transform + Eq. 3 and the phase passes
                st.accumulate(d_idx, d_off, 0, F, **com_kw)
                side.wait_stream(main_stream)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, n_com, det, scan, optics, dpc, com64=com64, phase=phase_dpc,
                                 ws=ws, d_status=status)
                st.finalize(phase=phase_ssb, T=T_ssb)
                main_stream.wait_stream(side)
            elif fused:
                st.oneshot(d_idx, d_off, phase=phase_ssb, T=T_ssb, **com_kw)
                stem.com_dpc(d_idx, d_off, 0, 0, det, scan, optics, dpc, com64=com64, phase=phase_dpc, ws=ws,
                             d_status=status)
            else:
                stem.com_dpc(d_idx, d_off, 0, F, det, scan, optics, dpc, com64=com64, phase=phase_dpc, ws=ws,
                             d_status=status)
                st.oneshot(d_idx, d_off, phase=phase_ssb, T=T_ssb)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        stem.check_status(status, "com_dpc")
        stem.check_status(st.status, "ssb_reconstruct")
        stem.trace_enable(trace)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(main_stream)
        for k in range(steps):
            step()
            ev[k + 1].record(main_stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        recs = stem.trace_records() if trace else {}
        stem.trace_enable(False)
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        out = {"elapsed": elapsed, "ms": elapsed / steps * 1e3, "median_ms": statistics.median(per),
               "min_ms": min(per), "recs": recs, "stats": st.stats()}
        if keep:
            out.update(phase=phase_ssb.clone(), T=T_ssb.clone(), st=st)
        else:
            del st
        return out

    # the FP32 step, both G modes, one stream and COM + DPC on a second stream; the fastest is the
    # headline (step times from untraced runs)
    modes = [args.g_mode] if args.g_mode != "auto" else ["recompute", "store"]
    schedules = {}
    ovs = {"both": (False, True), "serial": (False,), "overlapped": (True,)}[args.schedules]
    for m in modes:
        for ov in ovs:
            r = run(stem.STEM_FFT_FP32, G_MODES[m], args.steps, args.warmup, overlap=ov)
            schedules[f"{m}/{'overlapped' if ov else 'serial'}"] = r
            log(f"FP32 {m:9s} {'overlapped' if ov else 'serial':10s}: mean {r['ms']:.4f} ms, median "
                f"{r['median_ms']:.4f} ms, min {r['min_ms']:.4f} ms")
    head_key = min(schedules, key=lambda k: schedules[k]["ms"])
    # the library's default recompute scratch (64 MiB: several chunks of pixels), for comparison
    if not args.no_default_scratch:
        r = run(stem.STEM_FFT_FP32, stem.STEM_G_RECOMPUTE, args.steps, args.warmup, overlap=False, scratch_mib=0)
        schedules["recompute(64MiB)/serial"] = r
        log(f"FP32 recompute with the default 64 MiB scratch, serial: mean {r['ms']:.4f} ms ({r['stats'][3]} chunks)")
    head = schedules[head_key]
    head_mode, head_sched = head_key.split("/")
    head_overlap = head_sched == "overlapped"
    # kernel times of the headline mode from a traced run on one stream (each kernel's HIP-event time is
    # its own), keeping its outputs for the error against the oracle
    tr = run(stem.STEM_FFT_FP32, G_MODES[head_mode], args.steps, args.warmup, overlap=False, trace=True, keep=True)
    P, groups, sum_read, chunks = tr["stats"]
    n_k = tr["st"].n_k
    phi32, T32 = tr["phase"].cpu().numpy().reshape(ny, nx), tr["T"].cpu().numpy().reshape(ny, nx)
    del tr["st"]
    log(f"headline: {head_key} {head['ms']:.4f} ms/step, n_K={n_k}, pairs={P}, chunks={chunks}")

    geo = {"C": C, "F": F, "nk": n_k, "nx": nx, "ny": ny, "P": P, "d_bytes": 1, "sum_read": sum_read,
           "store": head_mode == "store"}
    kernels = {}
    for name, (n, ms) in sorted(tr["recs"].items(), key=lambda kv: -kv[1][1]):
        per = n / args.steps
        ms_step = ms / args.steps
        ab = algorithmic_bytes(name, geo)
        cnt = load_traffic(name, args.workload)
        kernels[name] = {"launches_per_step": per, "avg_us": round(ms / n * 1e3, 2), "us_per_step": round(ms_step * 1e3, 2),
                         "gbs": round(ab[0] / (ms_step * 1e-3) / 1e9, 1) if ab else None,
                         "gbs_with_D": round(ab[1] / (ms_step * 1e-3) / 1e9, 1) if ab else None,
                         "gbs_counted": round(cnt * per / (ms_step * 1e-3) / 1e9, 1) if cnt else None}
        log(f"  {name:18s} {per:4.1f} x {ms / n * 1e3:9.2f} us"
            + (f"  {ab[0] / 1e6:9.2f} MB  {ab[0] / (ms_step * 1e-3) / 1e9:8.1f} GB/s" if ab else ""))
    dom = max((k for k in kernels if algorithmic_bytes(k, geo)), key=lambda k: kernels[k]["us_per_step"])
    ab = algorithmic_bytes(dom, geo)
    t_step = kernels[dom]["us_per_step"] * 1e-6
    per_launch = kernels[dom]["launches_per_step"]
    cnt = load_traffic(dom, args.workload)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ab[0] / t_step / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ab[0] / t_step / 1e9 / HBM_PEAK_GBS, 4), "traffic": cnt,
                "bytes_per_launch": int(ab[0] / per_launch), "avg_launch_us": kernels[dom]["avg_us"],
                "with_D": {"bytes_per_launch": int(ab[1] / per_launch),
                           "achieved": round(ab[1] / t_step / 1e9, 1),
                           "frac": round(ab[1] / t_step / 1e9 / HBM_PEAK_GBS, 4)}}
    sb = step_bytes(geo)
    step_roof = {"bytes": sb, "achieved": round(sb / (head["ms"] * 1e-3) / 1e9, 1),
                 "frac": round(sb / (head["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"roofline {dom}: {roofline['achieved']} GB/s = {roofline['frac']} of peak "
        f"({roofline['with_D']['frac']} with D); whole step {step_roof['frac']}")

    # kernel times of the other G mode's one-shot step, traced on one stream
    other = "store" if head_mode == "recompute" else "recompute"
    ro = run(stem.STEM_FFT_FP32, G_MODES[other], args.steps, args.warmup, overlap=False, trace=True)
    other_kernels = {k: round(ms / n * 1e3, 2) for k, (n, ms) in ro["recs"].items()}
    log(f"{other} mode kernels (us per launch): {other_kernels}")

    def ssb_us(recs):
        return sum(ms for name, (n, ms) in recs.items() if not name.startswith(("com_", "dpc_"))) / args.steps * 1e3

    ssb32 = ssb_us(tr["recs"])
    variants = {}
    keep_split = {}
    if not args.no_split:
        for label, prec in (("bf16_split", stem.STEM_DFT_BF16_SPLIT), ("fp16_split", stem.STEM_DFT_FP16_SPLIT)):
            rv = run(prec, G_MODES[head_mode], args.steps, args.warmup, overlap=False, trace=True, keep=True)
            phi_v, T_v = rv["phase"].cpu().numpy().reshape(ny, nx), rv["T"].cpu().numpy().reshape(ny, nx)
            del rv["st"]
            ru = run(prec, G_MODES[head_mode], args.steps, args.warmup, overlap=head_overlap)
            # the stored double-overlap values of a stored-G FINALIZE (the G the sum uses)
            stv = stem.SsbState(det, scan, optics, stem.Ssb(prec, 0, stem.STEM_G_STORE, 8), device=dev)
            stv.oneshot(d_idx, d_off)
            poff = stv.region(stem.STEM_REGION_POFF).view(torch.int64)
            npg = int(poff[-1].item())
            keep_split[label] = {"phi": phi_v, "T": T_v,
                                 "pg": stv.region(stem.STEM_REGION_PG).view(torch.complex64)[:npg].cpu().numpy()}
            del stv
            sm = ssb_us(rv["recs"])
            variants[label] = {
                "ms_per_step": round(ru["ms"], 4), "median_ms": round(ru["median_ms"], 4),
                "value": round(C * args.steps / ru["elapsed"], 1),
                "speedup_vs_fp32_step": round(head["ms"] / ru["ms"], 3),
                "ssb_us": round(sm, 2), "speedup_vs_fp32_ssb": round(ssb32 / sm, 3), "speedup_target": 2.0,
                "phi_rel_l2_vs_fp32_path": float(f"{rel_l2(phi_v, phi32):.3e}"),
                "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in rv["recs"].items()},
            }
            log(f"{label}: {ru['ms']:.4f} ms/step (SSB {sm:.1f} us vs FP32 {ssb32:.1f} us)")

    def timed(fn):
        """(seconds for args.steps untraced calls of fn, kernel records of as many traced calls)"""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stem.trace_enable(True)
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        recs = stem.trace_records()
        stem.trace_enable(False)
        return el, recs

    extras = {}
    if not args.no_extras:
        # the same step with the aberrations of the aberrated workload corrected in Eq. 3
        opt_c = stem.Optics.from_values(wl.lam, wl.r_bf, wl.dk, C4_TRUE_ABERRATIONS)
        ra = run(stem.STEM_FFT_FP32, G_MODES[head_mode], args.steps, args.warmup, overlap=False, opt=opt_c, trace=True)
        rc = run(stem.STEM_FFT_FP32, G_MODES[head_mode], args.steps, args.warmup, overlap=head_overlap, opt=opt_c)
        extras["aberration_corrected"] = {
            "workload": "scan1024 with the probe aberrations C1..C3 of the aberrated workload corrected in Eq. 3",
            "ms_per_step": round(rc["ms"], 4), "value": round(C * args.steps / rc["elapsed"], 1),
            "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in ra["recs"].items()}}
        log(f"aberration-corrected step: {rc['ms']:.4f} ms")

        # interactive refocus from the stored double-overlap values; the panel of G (Fig. 2)
        st = stem.SsbState(det, scan, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, stem.STEM_G_STORE, 8), device=dev)
        st.oneshot(d_idx, d_off, phase=phase_ssb)
        c_new = tuple(0.5 * v for v in C4_TRUE_ABERRATIONS)
        for _ in range(args.warmup):
            st.refocus(c=c_new, phase=phase_ssb)
        el_r, rr = timed(lambda: st.refocus(c=c_new, phase=phase_ssb))
        torch.cuda.synchronize()
        ref_stats = st.stats()
        n_r, ms_r = rr.get("ssb_reduce", (1, float("nan")))
        extras["refocus"] = {"workload": "scan1024, stored double-overlap G, aberrated coefficients",
                             "ms": round(el_r / args.steps * 1e3, 4),
                             "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in rr.items()},
                             "sum_bytes_read": ref_stats[2],
                             "sum_gbs": round(ref_stats[2] / (ms_r / n_r * 1e-3) / 1e9, 1),
                             "plan_bytes": 8 * P + 28 * F,
                             "plan_frac": round((8 * P + 28 * F) / (el_r / args.steps) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"refocus: {el_r / args.steps * 1e3:.4f} ms ({extras['refocus']['kernels_us']})")
        qs9 = [(my, mx) for my in (1, 2, 3) for mx in (1, 2, 3)]
        st.g_panel(qs9)
        _, rp = timed(lambda: st.g_panel(qs9))
        n_, ms_ = rp["g_panel"]
        extras["g_panel"] = {"workload": "scan1024, G at nine scan frequencies as binned detector images",
                             "from_row_transform_us": round(ms_ / n_ * 1e3, 2)}
        del st
        stg = {}
        for m in ("recompute", "store"):
            stg[m] = stem.ssb_state_bytes(det, scan, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, G_MODES[m], 8))
        extras["state_bytes"] = stg

        # Eq. 3 as a batched complex matrix product (the remark after Eq. 3): per column mx,
        # T(my) = sum_K A(K, my) G(K, my) is the diagonal of A^T G, a (Ny x n_K) by (n_K x Ny)
        # product per column.  A lower bound on that route: torch's batched complex64 product for a
        # sample of columns (operands contiguous, their construction not timed), scaled to all
        # Nx/2 + 1 columns, against the fused column sum that also transforms the columns.
        ncol = 16
        ga = torch.randn(ncol, scan.ny, n_k, dtype=torch.complex64, device=dev).contiguous()
        gb = torch.randn(ncol, n_k, scan.ny, dtype=torch.complex64, device=dev).contiguous()
        for _ in range(2):
            torch.bmm(ga, gb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.bmm(ga, gb)
        e1.record()
        torch.cuda.synchronize()
        bmm_us = e0.elapsed_time(e1) / 5 * 1e3 * (scan.nx // 2 + 1) / ncol
        flops = 8.0 * (scan.nx // 2 + 1) * scan.ny * scan.ny * n_k
        extras["eq3_as_gemm"] = {"workload": f"scan1024 geometry: {scan.nx // 2 + 1} columns of a ({scan.ny} x {n_k}) by "
                                             f"({n_k} x {scan.ny}) complex product, {ncol} timed and scaled",
                                 "gemm_us": round(bmm_us, 1), "gemm_tflops": round(flops / (bmm_us * 1e-6) / 1e12, 1),
                                 "fused_sum_us": kernels.get("ssb_yreduce", {}).get("avg_us")}
        log(f"Eq. 3 as a batched complex product: {bmm_us:.0f} us for all columns ({flops / 1e12:.2f} TFLOP)")
        del ga, gb

        # differentiation workload: forward + adjoint of -Var(phi) w.r.t. the 8 coefficients
        wl4 = WORKLOADS["aberrated512"]
        d4 = simulate(wl4, device=dev)
        torch.cuda.synchronize()
        H4, W4 = wl4.det
        det4 = stem.Det(W4, H4, W4 // 2, H4 // 2, wl4.bin)
        scan4 = stem.Scan(wl4.scan[0], wl4.scan[1], wl4.step)
        c4 = tuple(v * (1 + 0.25 * (-1) ** j) for j, v in enumerate(wl4.aberr))
        opt4 = stem.Optics.from_values(wl4.lam, wl4.r_bf, wl4.dk, c4)
        ph4 = torch.empty(wl4.n_frames, dtype=torch.float32, device=dev)
        adj = {"workload": f"aberrated512: {wl4.name}", "n_k": int(stem.ssb_num_pixels(det4, opt4))}
        for m in ("recompute", "store"):
            st = stem.SsbState(det4, scan4, opt4, stem.Ssb(stem.STEM_FFT_FP32, 0, G_MODES[m], 8, args.scratch_mib),
                               device=dev)
            st.accumulate(d4.idx, d4.off, 0, wl4.n_frames)

            def fb():
                st.finalize(phase=ph4)
                gbar = (-(2.0 / ph4.numel()) * (ph4 - ph4.mean())).contiguous()
                return st.backward(gbar)

            for _ in range(args.warmup):
                fb()
            el_a, ra = timed(fb)
            adj[m] = {"forward_plus_backward_ms": round(el_a / args.steps * 1e3, 4),
                      "state_bytes": stem.ssb_state_bytes(det4, scan4, opt4, stem.Ssb(stem.STEM_FFT_FP32, 0, G_MODES[m], 8)),
                      "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in ra.items()}}
            log(f"aberrated512 forward + adjoint ({m}): {el_a / args.steps * 1e3:.3f} ms {adj[m]['kernels_us']}")
            del st
        extras["adjoint"] = adj
        del d4

        # virtual detectors from the same events: bright-field + annular dark-field images, PACBED
        vd = torch.empty(2 * F, dtype=torch.int32, device=dev)
        pac = torch.zeros(W * H, dtype=torch.int32, device=dev)
        r_in, r_out = [0.0, 1.2 * wl.r_bf], [wl.r_bf, 4.0 * wl.r_bf]

        def detectors():
            stem.virtual_annular(d_idx, d_off, 0, F, det, scan, r_in, r_out, vd, d_status=status)
            pac.zero_()
            stem.sum_frames(d_idx, d_off, 0, F, det, pac, d_status=status)

        for _ in range(args.warmup):
            detectors()
        el_v, rv = timed(detectors)
        stem.check_status(status, "virtual detectors")
        kv = {k: round(ms / n * 1e3, 2) for k, (n, ms) in rv.items()}
        extras["virtual_detectors"] = {
            "workload": "scan1024: bright field [0, r_bf) and annular dark field [1.2, 4) r_bf per frame; "
                        "sum of all frames",
            "ms": round(el_v / args.steps * 1e3, 4), "kernels_us": kv,
            "annular_events_per_s": round(C / (kv.get("virtual_annular", float("nan")) * 1e-6), 1)}
        log(f"virtual detectors: {el_v / args.steps * 1e3:.3f} ms {kv}")
        del vd, pac
        # run-length form of the same events re-coded to linear indices
        from gen import run_length_form
        dist = run_length_form(d_idx, d_off)
        dec = torch.empty_like(d_idx)
        for _ in range(args.warmup):
            stem.eer_decode_rle(dist, d_off, 0, F, det, dec, d_status=status)
        _, rr = timed(lambda: stem.eer_decode_rle(dist, d_off, 0, F, det, dec, d_status=status))
        stem.check_status(status, "run-length decoding")
        assert torch.equal(dec, d_idx)
        n_, ms_ = rr["decode_rle"]
        extras["decode_rle"] = {"workload": "scan1024 events in run-length form", "us": round(ms_ / n_ * 1e3, 2),
                                "events_per_s": round(C / (ms_ / n_ * 1e-3), 1)}
        log(f"run-length decoding: {ms_ / n_ * 1e3:.1f} us")
        del dist, dec

        # end to end from pinned host memory: 16 chunks of 64 scan rows; the copy (and validation) of
        # chunk k+1 on a copy stream overlaps COM + binning (+ row transform with stored G) of chunk k
        h_idx = d_idx.cpu().pin_memory()
        h_off = d_off.cpu().pin_memory()
        s_idx = torch.empty_like(d_idx)
        s_off = torch.empty_like(d_off)
        copy = torch.cuda.Stream(device=dev)  # default priority
        st = stem.SsbState(det, scan, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, G_MODES[head_mode], 8, args.scratch_mib),
                           device=dev)
        rows = 64
        offs = d_off.cpu().numpy()
        chunks_h = [(r0 * nx, rows * nx, int(offs[r0 * nx]), int(offs[(r0 + rows) * nx])) for r0 in range(0, ny, rows)]
        ready = [torch.cuda.Event() for _ in chunks_h]
        h2d_status = stem.status_tensor(dev)

        def streamed(compute=True):
            copy.wait_stream(main_stream)
            for j, (f0, nf, e0, e1) in enumerate(chunks_h):
                with torch.cuda.stream(copy):
                    stem.eer_load_csr(h_idx[e0:e1], h_off[f0:f0 + nf + 1], f0, nf, e1 - e0, det, s_idx, s_off,
                                      d_status=h2d_status)
                    ready[j].record(copy)
                if compute:
                    main_stream.wait_event(ready[j])
                    last = j == len(chunks_h) - 1
                    stem.com_dpc(s_idx, s_off, f0, nf, det, scan, optics, dpc, com64=com64,
                                 phase=phase_dpc if last else None, ws=ws, d_status=status)
                    st.accumulate(s_idx, s_off, f0, nf)
            main_stream.wait_stream(copy)
            if compute:
                st.finalize(phase=phase_ssb)

        res = {}
        for label, comp in (("copy_only", False), ("end_to_end", True)):
            for _ in range(2):
                streamed(comp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                streamed(comp)
            torch.cuda.synchronize()
            res[label] = (time.perf_counter() - t0) / reps * 1e3
        stem.check_status(h2d_status, "streamed ingest")
        st.g_panel(qs9)
        _, rp = timed(lambda: st.g_panel(qs9))
        n_, ms_ = rp["g_panel"]
        extras["g_panel"][f"{head_mode}_mode_us"] = round(ms_ / n_ * 1e3, 2)
        assert torch.equal(s_idx, d_idx) and torch.equal(s_off, d_off)
        host_bytes = 4 * C + 8 * (F + len(chunks_h))
        extras["streamed"] = {"workload": "scan1024 in 16 chunks of 64 scan rows from pinned host memory",
                              "end_to_end_ms": round(res["end_to_end"], 3),
                              "events_per_s": round(C / (res["end_to_end"] * 1e-3), 1),
                              "positions_per_s": round(F / (res["end_to_end"] * 1e-3), 1),
                              "copy_only_ms": round(res["copy_only"], 3),
                              "h2d_gbs": round(host_bytes / (res["copy_only"] * 1e-3) / 1e9, 1)}
        log(f"streamed from host: end to end {res['end_to_end']:.3f} ms, copies alone {res['copy_only']:.3f} ms")
        del st, h_idx, h_off, s_idx, s_off

    # what plain streaming kernels reach on this HBM (torch's copy and fill of 1 GiB), for context
    hbm_ref = {}
    a = torch.empty((1 << 30) // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for label, fn, nbytes in (("copy", lambda: b.copy_(a), 2 << 30), ("fill", lambda: b.fill_(2.0), 1 << 30)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        hbm_ref[f"{label}_gbs"] = round(nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    hbm_ref["dominant_frac_of_copy"] = round(roofline["achieved"] / hbm_ref["copy_gbs"], 3)
    log(f"HBM reference: copy {hbm_ref['copy_gbs']} GB/s, fill {hbm_ref['fill_gbs']} GB/s")

    cpu = None
    errors = {}
    if pool is not None:
        idx_np = d_idx.cpu().numpy()
        off_np = d_off.cpu().numpy()
        del data
        torch.cuda.empty_cache()
        t1, parts1, ref = oracle_single(idx_np, off_np, wl)
        log(f"oracle, 1 thread: {t1:.1f} s per step -> {C / t1:.3e} events/s")
        tn, partsn, phin = oracle_parallel(pool, n_workers, idx_np, off_np, wl)
        log(f"oracle, {n_workers} processes: {tn:.1f} s per step -> {C / tn:.3e} events/s")
        pool.close()
        pool.join()
        cpu = {"value": round(C / tn, 1), "unit": "events/s", "cores": n_workers, "kind": "oracle",
               "sample": (f"the whole workload, one step: COM + DPC of all {F} frames, binning, scan DFT of all "
                          f"{len(ref['kc'])} pixels, Eq. 3 sum, phase; FP64 numpy oracle in {n_workers} worker "
                          "processes (frame shards for COM and binning, pixel shards for the transform and sum)"),
               "seconds": round(tn, 2), "stage_seconds": {k: round(v, 3) for k, v in partsn.items()},
               "positions_per_s": round(F / tn, 1),
               "single_thread": {"value": round(C / t1, 1), "cores": 1, "seconds": round(t1, 2),
                                 "stage_seconds": {k: round(v, 3) for k, v in parts1.items()}},
               "host_cpus": os.cpu_count()}
        assert rel_l2(phin, ref["phi"]) < 1e-10  # the sharded run computes the same phase
        # every output of the GPU runs against the FP64 oracle
        pg_ref = oracle_pruned_values(ref["G"], ref["kc"], wl)
        errors["fp32"] = {"T": rel_l2(T32, ref["T"]), "phi": rel_l2(phi32, ref["phi"])}
        for label, o in keep_split.items():
            errors[label] = {"G": rel_l2(o["pg"], pg_ref), "T": rel_l2(o["T"], ref["T"]),
                             "phi": rel_l2(o["phi"], ref["phi"])}
            variants[label]["rel_l2_vs_fp64_oracle"] = {k: float(f"{v:.3e}") for k, v in errors[label].items()}
        log(f"errors against the oracle: {errors}")

    out = {
        "metric": METRIC,
        "value": round(C * args.steps / head["elapsed"], 1),
        "unit": "events/s",
        "positions_per_s": round(F * args.steps / head["elapsed"], 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "median_ms": round(head["median_ms"], 4),
        "min_ms": round(head["min_ms"], 4),
        "schedule": head_key,
        "schedules_ms": {k: {"mean": round(v["ms"], 4), "median": round(v["median_ms"], 4),
                             "min": round(v["min_ms"], 4)} for k, v in schedules.items()},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.name}", "scan": [ny, nx], "detector": [H, W],
                   "bin": wl.bin, "mean_e_per_frame": wl.mean_e, "events": C, "frames": F, "n_k": n_k,
                   "double_overlap_pairs": P,
                   "ssb_path": (f"FP32 FFT, G mode {head_mode} ({chunks} pixel chunks), fused column transform + "
                                "Eq. 3; no aberrations, so the phase factors of Eq. 3 are exactly 1 (the "
                                "aberration-corrected step is reported beside it)"),
                   "com": ("formed by the binning pass (ssb_reconstruct_com); com_dpc integrates only"
                           if args.fused_com else "own pass over the events (com_dpc)"),
                   "parallelism": "single GPU"},
        "kernels": kernels,
        f"kernels_us_{other}_mode": other_kernels,
        "ssb_us_fp32": round(ssb32, 2),
        "fp32_rel_l2_vs_fp64_oracle": {k: float(f"{v:.3e}") for k, v in errors.get("fp32", {}).items()},
        "precision_variants": variants,
        **extras,
        "roofline": roofline,
        "step_roofline": step_roof,
        "hbm_reference": hbm_ref,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
