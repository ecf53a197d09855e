#!/usr/bin/env python
"""Throughput of the event-based phase-contrast path on one MI355X.

One step = the whole hot path over one synthetic acquisition already resident in HBM:
centre of mass of every frame + DPC integration (com_dpc), then the single-sideband
reconstruction (ssb_reconstruct, one shot: binning, scan transform, double-overlap sum,
phase image).  Reported: events/s (value) and scan positions/s, with the per-kernel
roofline of the dominant kernel, the split-precision scan-DFT variants, and the FP64 CPU oracle
timed on the same workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--workload scan1024]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/s + scan positions/s, COM-DPC+SSB; BF16-split vs FP32 at <=1e-4 error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(name, g):
    """Bytes a kernel must move per launch (see the data-layout section of the design notes).

    g: dict with C (events), F (frames), nk, nx, ny, P (double-overlap pairs), d_bytes."""
    C, F, nk, nx, ny, P = g["C"], g["F"], g["nk"], g["nx"], g["ny"], g["P"]
    nh = nx // 2 + 1
    X = nk * nh * ny * 8  # row-transformed cube, complex64
    table = {
        "com_moments": 4 * C + 8 * (F + 1) + 16 * F,           # events, offsets, COM (FP64, 2 planes)
        "bin_densify": 4 * C + 8 * (F + 1) + nk * F * g["d_bytes"],
        "bin_com": 4 * C + 8 * (F + 1) + nk * F * g["d_bytes"] + 16 * F,  # binning + COM (FP64) out
        "xstage_fft": nk * F * g["d_bytes"] + X,               # D in, X out
        "ystage_fft": 2 * X,                                    # X in, G out (in place)
        "ssb_yreduce": X + 8 * F * g["groups"],                # X in, partial T per pixel group out
        "ssb_reduce": 8 * P + 8 * F,                            # G on the double-overlap pairs, T out
        "phase_fft": 8 * F * (1 + g["groups"]) // 2 + 8 * F,  # the two passes averaged: partial sums in, T out
        # DPC: COM planes (FP64) in, half spectra Gx, Gy out; both in, half-spectrum result out;
        # that in, the phase image (FP32) out
        "dpc_rows": 16 * F + 2 * 8 * nh * ny,
        "dpc_cols": 2 * 8 * nh * ny + 8 * nh * ny,
        "dpc_fft": 8 * nh * ny + 4 * F,
    }
    return table.get(name)


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
    "stem::k_bin<unsigned char, true, true>": "bin_com",
    "stem::k_xstage<stem::XfFft<1024>, unsigned char>": "xstage_fft",
    "stem::k_yreduce<stem::XfFft<1024>, true>": "ssb_yreduce",
    "stem::k_dpc_cols<1024, 4>": "dpc_cols",
}


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
    import statistics
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

    val = per_kernel(rd, "stem::k_validate", rbytes)[0]
    read_factor = val / (4 * C + 8 * (F + 1))
    copies = [c["WRITE_SIZE"] * 1024 for (_, k, g), c in wr.items() if "direct_copy" in k and g == 33546240]
    write_factor = statistics.mean(copies) / (1 << 30)
    rec = {"_note": summarize_profile.__doc__.split("\n\n")[1].replace("\n    ", " ").strip(),
           "read_factor": round(read_factor, 5), "write_factor": round(write_factor, 5)}
    sha = source_sha()
    lines = ["| Kernel | Trace name | Dispatches | FETCH_SIZE (MB, raw) | Reads (MB, calibrated) "
             "| Writes (MB, calibrated) |", "|---|---|---:|---:|---:|---:|"]
    for kname, tname in PROFILED.items():
        r, n = per_kernel(rd, kname, rbytes)
        w, _ = per_kernel(wr, kname, lambda c: c["WRITE_SIZE"] * 1024)
        fs, _ = per_kernel(fetch, kname, lambda c: c["FETCH_SIZE"] * 1024)
        if r is None or w is None:
            continue
        r, w = r / read_factor, w / write_factor
        rec[f"{tname}@{workload}"] = {"bytes_per_launch": int(r + w), "read_bytes": int(r), "write_bytes": int(w),
                                      "source_sha": sha}
        lines.append(f"| `{kname}` | {tname} | {n} | {fs / 1e6 if fs else float('nan'):.1f} | {r / 1e6:.1f} "
                     f"| {w / 1e6:.1f} |")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(f"C = {C}, F = {F}; read factor {read_factor:.5f} (k_validate), write factor {write_factor:.5f} "
          f"(1 GiB copy, {len(copies)} dispatches); sources sha {sha}\n")
    print("\n".join(lines))
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


def cpu_baseline(idx, off, wl):
    """The FP64 oracle on the host over the whole workload (COM + DPC, binning, scan DFT,
    Eq. 3 sum, phase), each stage timed; numpy runs these single-threaded."""
    from oracle import dpc as odpc
    from oracle import eer as oeer
    from oracle import ssb as ossb

    H, W = wl.det
    ny, nx = wl.scan
    F = wl.n_frames
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
    T, _ = ossb.ssb_sum(G, kc, wl.step, wl.dk, wl.lam, wl.r_bf, wl.aberr)
    t["ssb_sum"] = time.perf_counter() - t0
    del G
    t0 = time.perf_counter()
    ossb.phase_from_T(T)
    t["phase"] = time.perf_counter() - t0
    total = sum(t.values())
    return total, t, (f"FP64 numpy oracle, 1 thread, the whole workload: COM + DPC on all {F} frames, binning, "
                      f"scan DFT of all {len(kc)} pixels, Eq. 3 sum, phase IFFT (one step, no scaling)")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scan1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision scan-DFT variants")
    ap.add_argument("--no-extras", action="store_true", help="skip the refocus and adjoint timings")
    ap.add_argument("--com-beside", choices=("finalize", "binning"), default="finalize",
                    help="where COM runs on the second stream: beside FINALIZE (with DPC), or from the start "
                         "of the step beside the binning (DPC still beside FINALIZE)")
    ap.add_argument("--fused-com", action="store_true",
                    help="centre of mass formed by the binning pass (ssb_reconstruct_com) instead of its own "
                         "pass over the events on the second stream")
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

    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    side = torch.cuda.Stream(device=dev)  # default priority

    def run(precision, steps, warmup, overlap=True, opt=optics, trace=False):
        """Times `steps` whole steps with the given scan-DFT precision; returns
        (elapsed s, kernel trace, SSB phase, SsbState).  With overlap, COM + DPC run on a second
        stream concurrently with the second half of the SSB reconstruction (FINALIZE after
        ACCUMULATE over all frames, the same work as ONESHOT; the two share only the read-only
        events).  With trace, a HIP event pair brackets every kernel (per-kernel times); the event
        records add queue packets between kernels, so step times are taken without them."""
        st = stem.SsbState(det, scan, opt, stem.Ssb(precision, 0, stem.STEM_G_RECOMPUTE, 8), device=dev)
        main = torch.cuda.current_stream(dev)

        # com_dpc reads the events itself on the second stream (beside FINALIZE); with --fused-com
        # the binning pass forms the centre of mass (one read of the events, on the critical path)
        # and com_dpc only integrates (n_frames = 0)
        fused = args.fused_com
        com_kw = {"com64": com64} if fused else {}
        n_com = 0 if fused else F

        early_com = args.com_beside == "binning" and not fused

        def step():
            if overlap and early_com:
                # COM reads the events beside the binning (which reads them too); DPC waits for it and
                # for the row transform, then runs beside FINALIZE
                side.wait_stream(main)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, F, det, scan, com64=com64, d_status=status)
                st.accumulate(d_idx, d_off, 0, F)
                side.wait_stream(main)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, 0, det, scan, optics, dpc, com64=com64, phase=phase_dpc,
                                 ws=ws, d_status=status)
                st.finalize(phase=phase_ssb)
                main.wait_stream(side)
            elif overlap:
                # binning (+ COM) and the row transform first; DPC (latency-bound) then runs beside
                # the VALU-bound column transform + Eq. 3 and the phase passes
                st.accumulate(d_idx, d_off, 0, F, **com_kw)
                side.wait_stream(main)
                with torch.cuda.stream(side):
                    stem.com_dpc(d_idx, d_off, 0, n_com, det, scan, optics, dpc, com64=com64, phase=phase_dpc,
                                 ws=ws, d_status=status)
                st.finalize(phase=phase_ssb)
                main.wait_stream(side)
            elif fused:
                st.oneshot(d_idx, d_off, phase=phase_ssb, **com_kw)
                stem.com_dpc(d_idx, d_off, 0, 0, det, scan, optics, dpc, com64=com64, phase=phase_dpc, ws=ws,
                             d_status=status)
            else:
                stem.com_dpc(d_idx, d_off, 0, F, det, scan, optics, dpc, com64=com64, phase=phase_dpc, ws=ws,
                             d_status=status)
                st.oneshot(d_idx, d_off, phase=phase_ssb)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        stem.check_status(status, "com_dpc")
        stem.check_status(st.status, "ssb_reconstruct")
        stem.trace_enable(trace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        recs = stem.trace_records() if trace else {}
        stem.trace_enable(False)
        return elapsed, recs, phase_ssb.clone(), st

    # kernel times from a traced serial run (no overlap: each kernel's HIP-event time is its own),
    # step times from untraced runs
    _, recs, phi32, st = run(stem.STEM_FFT_FP32, args.steps, args.warmup, overlap=False, trace=True)
    del st
    el_serial, _, _, st = run(stem.STEM_FFT_FP32, args.steps, args.warmup, overlap=False)
    del st
    elapsed, _, _, st = run(stem.STEM_FFT_FP32, args.steps, args.warmup)
    ms_per_step = elapsed / args.steps * 1e3
    log(f"serial step {el_serial / args.steps * 1e3:.3f} ms, overlapped step {ms_per_step:.3f} ms")
    P, groups = st.stats()[:2]
    n_k = st.n_k
    del st
    log(f"{args.steps} steps in {elapsed:.4f} s ({ms_per_step:.3f} ms/step), n_K={n_k}, pairs={P}")

    geo = {"C": C, "F": F, "nk": n_k, "nx": nx, "ny": ny, "P": P, "d_bytes": 1, "groups": groups}
    kernels = {}
    for name, (n, ms) in sorted(recs.items(), key=lambda kv: -kv[1][1]):
        per = n / args.steps
        avg_ms = ms / n
        ab = algorithmic_bytes(name, geo)
        kernels[name] = {"launches_per_step": per, "avg_ms": round(avg_ms, 5),
                         "ms_per_step": round(ms / args.steps, 5),
                         "gbs": round(ab / (avg_ms * 1e-3) / 1e9, 1) if ab else None}
        log(f"  {name:16s} {per:4.1f} x {avg_ms * 1e3:9.2f} us"
            + (f"  {ab / 1e6:9.2f} MB  {ab / (avg_ms * 1e-3) / 1e9:8.1f} GB/s" if ab else ""))
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    ab = algorithmic_bytes(dom, geo)
    avg_s = kernels[dom]["avg_ms"] * 1e-3
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ab / avg_s / 1e9, 1) if ab else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ab / avg_s / 1e9 / HBM_PEAK_GBS, 4) if ab else None,
                "traffic": load_traffic(dom, args.workload), "bytes_per_launch": ab}

    def ssb_ms(r):
        return sum(ms for name, (n, ms) in r.items() if not name.startswith(("com_", "dpc_"))) / args.steps

    ssb32 = ssb_ms(recs)
    variants = {}
    if not args.no_split:
        for label, prec in (("bf16_split", stem.STEM_DFT_BF16_SPLIT), ("fp16_split", stem.STEM_DFT_FP16_SPLIT)):
            _, rv, phi, st = run(prec, args.steps, args.warmup, overlap=False, trace=True)  # kernel times
            del st
            el, _, _, st = run(prec, args.steps, args.warmup)                # overlapped step
            del st
            d = float((phi.double() - phi32.double()).norm() / phi32.double().norm())
            sm = ssb_ms(rv)
            variants[label] = {
                "ms_per_step": round(el / args.steps * 1e3, 4),
                "value": round(C * args.steps / el, 1),
                "speedup_vs_fp32_step": round(elapsed / el, 3),
                "ssb_ms": round(sm, 4),
                "speedup_vs_fp32_ssb": round(ssb32 / sm, 3),
                "phi_rel_l2_vs_fp32_path": float(f"{d:.3e}"),
                "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in rv.items()},
            }
            log(f"{label}: {el / args.steps * 1e3:.3f} ms/step (SSB {sm:.3f} ms vs FP32 {ssb32:.3f} ms), "
                f"phi vs FP32 path rel L2 {d:.2e}")

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

    # the same step with aberration correction (the general phase factors of Eq. 3 evaluated)
    extras = {}
    if not args.no_extras:
        opt_c = stem.Optics.from_values(wl.lam, wl.r_bf, wl.dk, C4_TRUE_ABERRATIONS)
        _, ra, _, st = run(stem.STEM_FFT_FP32, args.steps, args.warmup, overlap=False, opt=opt_c, trace=True)
        del st
        el_c, _, _, st = run(stem.STEM_FFT_FP32, args.steps, args.warmup, opt=opt_c)
        del st
        extras["aberration_corrected"] = {
            "workload": "scan1024 with the probe aberrations C1..C3 of the aberrated workload corrected in Eq. 3",
            "ms_per_step": round(el_c / args.steps * 1e3, 4), "value": round(C * args.steps / el_c, 1),
            "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in ra.items()}}
        log(f"aberration-corrected step: {el_c / args.steps * 1e3:.3f} ms, yreduce "
            f"{ra['ssb_yreduce'][1] / ra['ssb_yreduce'][0] * 1e3:.1f} us")

    # interactive refocus (stored G): Eq. 3 and the phase only, with new coefficients
    if not args.no_extras:
        st = stem.SsbState(det, scan, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, stem.STEM_G_STORE, 8), device=dev)
        st.oneshot(d_idx, d_off, phase=phase_ssb)
        c_new = tuple(0.5 * v for v in C4_TRUE_ABERRATIONS)
        for _ in range(args.warmup):
            st.refocus(c=c_new, phase=phase_ssb)
        el_r, rr = timed(lambda: st.refocus(c=c_new, phase=phase_ssb))
        # the panel of G at nine scan frequencies (Fig. 2), read from the stored G
        qs9 = [(my, mx) for my in (1, 2, 3) for mx in (1, 2, 3)]
        st.g_panel(qs9)
        torch.cuda.synchronize()
        stem.trace_enable(True)
        for _ in range(args.steps):
            st.g_panel(qs9)
        torch.cuda.synchronize()
        rp = stem.trace_records()
        stem.trace_enable(False)
        n_, ms_ = rp["g_panel"]
        extras["g_panel"] = {"workload": "scan1024, G at nine scan frequencies as binned detector images",
                             "stored_us": round(ms_ / n_ * 1e3, 2)}
        del st
        extras["refocus"] = {"workload": "scan1024, stored G, aberrated coefficients",
                             "ms": round(el_r / args.steps * 1e3, 4),
                             "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in rr.items()}}
        log(f"refocus: {el_r / args.steps * 1e3:.3f} ms")
        # differentiation workload: forward + adjoint of -Var(phi) w.r.t. the 8 coefficients
        wl4 = WORKLOADS["aberrated512"]
        d4 = simulate(wl4, device=dev)
        torch.cuda.synchronize()
        H4, W4 = wl4.det
        det4 = stem.Det(W4, H4, W4 // 2, H4 // 2, wl4.bin)
        scan4 = stem.Scan(wl4.scan[0], wl4.scan[1], wl4.step)
        c4 = tuple(v * (1 + 0.25 * (-1) ** j) for j, v in enumerate(wl4.aberr))
        opt4 = stem.Optics.from_values(wl4.lam, wl4.r_bf, wl4.dk, c4)
        st = stem.SsbState(det4, scan4, opt4, stem.Ssb(stem.STEM_FFT_FP32, 0, stem.STEM_G_RECOMPUTE, 8), device=dev)
        st.accumulate(d4.idx, d4.off, 0, wl4.n_frames)
        ph4 = torch.empty(wl4.n_frames, dtype=torch.float32, device=dev)

        def fb():
            st.finalize(phase=ph4)
            gbar = (-(2.0 / ph4.numel()) * (ph4 - ph4.mean())).contiguous()
            return st.backward(gbar)

        for _ in range(args.warmup):
            fb()
        torch.cuda.synchronize()
        el_a, ra = timed(fb)
        del st, d4
        extras["adjoint"] = {"workload": f"aberrated512: {wl4.name}", "n_k": int(stem.ssb_num_pixels(det4, opt4)),
                             "forward_plus_backward_ms": round(el_a / args.steps * 1e3, 4),
                             "kernels_us": {k: round(ms / n * 1e3, 2) for k, (n, ms) in ra.items()}}
        log(f"aberrated512 forward + adjoint: {el_a / args.steps * 1e3:.3f} ms")

    # virtual detectors from the same events: bright-field + annular dark-field images, PACBED
    if not args.no_extras:
        vd = torch.empty(2 * F, dtype=torch.int32, device=dev)
        pac = torch.zeros(W * H, dtype=torch.int32, device=dev)
        r_in, r_out = [0.0, 1.2 * wl.r_bf], [wl.r_bf, 4.0 * wl.r_bf]

        def detectors():
            stem.virtual_annular(d_idx, d_off, 0, F, det, scan, r_in, r_out, vd, d_status=status)
            pac.zero_()
            stem.sum_frames(d_idx, d_off, 0, F, det, pac, d_status=status)

        for _ in range(args.warmup):
            detectors()
        torch.cuda.synchronize()
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
        torch.cuda.synchronize()
        stem.trace_enable(True)
        for _ in range(args.steps):
            stem.eer_decode_rle(dist, d_off, 0, F, det, dec, d_status=status)
        torch.cuda.synchronize()
        rr = stem.trace_records()
        stem.trace_enable(False)
        stem.check_status(status, "run-length decoding")
        assert torch.equal(dec, d_idx)
        n_, ms_ = rr["decode_rle"]
        extras["decode_rle"] = {"workload": "scan1024 events in run-length form", "us": round(ms_ / n_ * 1e3, 2),
                                "events_per_s": round(C / (ms_ / n_ * 1e-3), 1)}
        log(f"run-length decoding: {ms_ / n_ * 1e3:.1f} us")
        del dist, dec

    # end to end from pinned host memory: 16 chunks of 64 scan rows; the copy (and validation) of
    # chunk k+1 on a copy stream overlaps COM + binning + row transform of chunk k
    if not args.no_extras:
        h_idx = d_idx.cpu().pin_memory()
        h_off = d_off.cpu().pin_memory()
        s_idx = torch.empty_like(d_idx)
        s_off = torch.empty_like(d_off)
        copy = torch.cuda.Stream(device=dev)  # default priority
        main = torch.cuda.current_stream(dev)
        st = stem.SsbState(det, scan, optics, stem.Ssb(stem.STEM_FFT_FP32, 0, stem.STEM_G_RECOMPUTE, 8), device=dev)
        rows = 64
        offs = d_off.cpu().numpy()
        chunks = [(r0 * nx, rows * nx, int(offs[r0 * nx]), int(offs[(r0 + rows) * nx])) for r0 in range(0, ny, rows)]
        ready = [torch.cuda.Event() for _ in chunks]
        h2d_status = stem.status_tensor(dev)

        def streamed(compute=True):
            copy.wait_stream(main)
            for j, (f0, nf, e0, e1) in enumerate(chunks):
                with torch.cuda.stream(copy):
                    stem.eer_load_csr(h_idx[e0:e1], h_off[f0:f0 + nf + 1], f0, nf, e1 - e0, det, s_idx, s_off,
                                      d_status=h2d_status)
                    ready[j].record(copy)
                if compute:
                    main.wait_event(ready[j])
                    last = j == len(chunks) - 1
                    stem.com_dpc(s_idx, s_off, f0, nf, det, scan, optics, dpc, com64=com64,
                                 phase=phase_dpc if last else None, ws=ws, d_status=status)
                    st.accumulate(s_idx, s_off, f0, nf)
            main.wait_stream(copy)
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
        if "g_panel" in extras:
            # the same panel computed from the row-transformed cube (G recomputed)
            stem.trace_enable(True)
            for _ in range(args.steps):
                st.g_panel(qs9)
            torch.cuda.synchronize()
            rp = stem.trace_records()
            stem.trace_enable(False)
            n_, ms_ = rp["g_panel"]
            extras["g_panel"]["recomputed_us"] = round(ms_ / n_ * 1e3, 2)
            log(f"g panel (9 frequencies): stored {extras['g_panel']['stored_us']} us, "
                f"recomputed {extras['g_panel']['recomputed_us']} us")
        assert torch.equal(s_idx, d_idx) and torch.equal(s_off, d_off)
        host_bytes = 4 * C + 8 * (F + len(chunks))
        extras["streamed"] = {"workload": "scan1024 in 16 chunks of 64 scan rows from pinned host memory",
                              "end_to_end_ms": round(res["end_to_end"], 3),
                              "events_per_s": round(C / (res["end_to_end"] * 1e-3), 1),
                              "positions_per_s": round(F / (res["end_to_end"] * 1e-3), 1),
                              "copy_only_ms": round(res["copy_only"], 3),
                              "h2d_gbs": round(host_bytes / (res["copy_only"] * 1e-3) / 1e9, 1)}
        log(f"streamed from host: end to end {res['end_to_end']:.3f} ms, copies alone {res['copy_only']:.3f} ms "
            f"({host_bytes / (res['copy_only'] * 1e-3) / 1e9:.1f} GB/s)")
        del st, h_idx, h_off, s_idx, s_off

    # what plain streaming kernels reach on this HBM (torch's copy and fill of 1 GiB), for context
    # beside the roofline fraction: the x-stage's traffic is 80% writes
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
    hbm_ref["dominant_frac_of_copy"] = (round(roofline["achieved"] / hbm_ref["copy_gbs"], 3)
                                        if roofline["achieved"] else None)
    log(f"HBM reference: copy {hbm_ref['copy_gbs']} GB/s, fill {hbm_ref['fill_gbs']} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        idx_np = d_idx.cpu().numpy()
        off_np = d_off.cpu().numpy()
        total, parts, sample = cpu_baseline(idx_np, off_np, wl)
        cpu = {"value": round(C / total, 1), "unit": "events/s", "cores": 1, "kind": "oracle", "sample": sample,
               "seconds": round(total, 2), "stage_seconds": {k: round(v, 3) for k, v in parts.items()}}
        log(f"cpu oracle {total:.1f} s per step -> {C / total:.3e} events/s")

    out = {
        "metric": METRIC,
        "value": round(C * args.steps / elapsed, 1),
        "unit": "events/s",
        "positions_per_s": round(F * args.steps / elapsed, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_serial": round(el_serial / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.name}", "scan": [ny, nx], "detector": [H, W],
                   "bin": wl.bin, "mean_e_per_frame": wl.mean_e, "events": C, "frames": F, "n_k": n_k,
                   "double_overlap_pairs": P, "ssb_path": "FP32 FFT, fused column transform + sum (G recomputed); no aberrations, so the "
                                   "phase factors of Eq. 3 are exactly 1 (the aberration-corrected step is "
                                   "reported beside it)",
                   "com": ("formed by the binning pass (ssb_reconstruct_com); com_dpc integrates only"
                           if args.fused_com else "own pass over the events (com_dpc) on the second stream"),
                   "parallelism": "single GPU"},
        "kernels": kernels,
        "ssb_ms_fp32": round(ssb32, 4),
        "precision_variants": variants,
        **extras,
        "roofline": roofline,
        "hbm_reference": hbm_ref,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
