#!/usr/bin/env python3
"""Benchmark: FPSA vs source-iteration time to solution at a 1e-8 stopping
test, and cell-angle updates/s, on one MI355X.

Workload (srk_slab_2000): homogeneous 100 mfp slab, 2000 LD cells, S_64
Gauss-Legendre, screened-Rutherford scattering eta = 1e-5 expanded to
L = 63, c = 0.999, uniform source q_n = 1, vacuum boundaries, FP64.

One step = one FPSA (WFD Laplacian) solve from phi^0 = 0 until
max|phi^{m+1} - phi^m| <= 1e-8: every iteration runs the scattering source,
the LD sweep, the moments, the Fokker-Planck correction and the stopping
test.  The factorisation of the Fokker-Planck operator is setup (done once,
untimed, as in the paper's timings).  Source iteration and FPSA with the MPD
Laplacian are timed beside it on the same handle type and reported in the
same JSON line.

value = cell-angle updates/s of the timed FPSA steps
      = iterations x cells x angles / seconds per solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-angle updates/s; solve time FPSA vs SI at 1e-8 residual (1 GPU)"
HBM_PEAK_GBS = 8000.0
# counter summaries: the single-slab FP64 kernels (srk_slab_2000) and the
# batched FP32 kernels (batch4096), each valid while its kernel sources hash
# to the value recorded in it
TRAFFIC_SETS = {
    "fpsa": ("profiles/fpsa_wfd_srk_slab_2000_traffic.txt",
             ("paper_1907_13013_amd/csrc/sn_kernels.hip", "paper_1907_13013_amd/csrc/sn_kernels.hpp")),
    "batch": ("profiles/batched_kernels_batch4096_traffic.txt",
              ("paper_1907_13013_amd/csrc/sn_batch.hip", "paper_1907_13013_amd/csrc/sn_batch.hpp")),
}
# kernels each counter summary covers
SET_KERNELS = {
    "fpsa": ("gemm_fp_source", "gemm_fp_update", "sweep_aggregate", "sweep_scan", "sweep_apply", "stopping_test",
             "fp_matvec", "fp_chain", "fp_carry", "fp_fixup", "exit_flux"),
    "batch": ("sweep_batch_dm", "sweep_batch_f32", "src_batch_p<128>", "mom_batch_p<128>", "src_batch_p<64>",
              "mom_batch_p<64>", "src_batch_p<32>", "mom_batch_p<32>", "fused_scan",
              *(f"fused_{k}{s}<{w}>" for s in ("", "_sp") for w in (128, 64, 32) for k in ("aggregate", "apply"))),
}
# launches per iteration of each fused pass instance on the 4096-slab batch
# (the 32-wide kernels also run the N = 16 class)
FUSED_LAUNCHES = {128: 1, 64: 1, 32: 2}
# substrings of the rocprofv3 kernel names of the timed kernel identities
# (the two GEMM instances of the correction are told apart by their K-chunk
# count on the 2000-cell S_64 workload: <2> forms the Fokker-Planck source
# from 2(L+1) = 128 moments, <3> the update from 128 moments and 64 inflows)
ROCPROF_NAME = {"gemm_fp_source": "snfpsa::gemm_f64_mfma<2>", "gemm_fp_update": "snfpsa::gemm_f64_mfma<3>",
                "sweep_aggregate": "snfpsa::sweep_aggregate",
                "sweep_scan": "snfpsa::sweep_scan_carry", "sweep_apply": "snfpsa::sweep_apply",
                "stopping_test": "snfpsa::stopping_test", "fp_matvec": "snfpsa::fp_matvec",
                "fp_chain": "snfpsa::fp_chain", "fp_carry": "snfpsa::fp_carry",
                "fp_fixup": "snfpsa::fp_fixup", "exit_flux": "snfpsa::exit_flux",
                "sweep_batch_dm": "snfpsa::sweep_batch_dm", "sweep_batch_f32": "snfpsa::sweep_batch_f32",
                # persistent FP32 class GEMMs of the batched solve (<32> also runs the W = 16 classes)
                "src_batch_p<128>": "snfpsa::src_batch_p<128, float>", "mom_batch_p<128>": "snfpsa::mom_batch_p<128>",
                "src_batch_p<64>": "snfpsa::src_batch_p<64, float>", "mom_batch_p<64>": "snfpsa::mom_batch_p<64>",
                "src_batch_p<32>": "snfpsa::src_batch_p<32, float>", "mom_batch_p<32>": "snfpsa::mom_batch_p<32>",
                # fused iteration: aggregate / apply passes per width; the last template argument is
                # the source's BF16 pieces (FP32 handles: 3, or 0 = FP32 MFMA at 32 wide; split: 2)
                "fused_scan": "snfpsa::fused_scan",
                **{f"fused_{k}{s}<{w}>": f"snfpsa::fused_tile<{w}, {'true' if k == 'apply' else 'false'}, "
                                          f"{2 if s else (0 if w == 32 else 3)}>"
                   for s in ("", "_sp") for w in (128, 64, 32) for k in ("aggregate", "apply")}}


def kernel_source_hash(which: str = "fpsa") -> str:
    """Hash of the code of a kernel set: its sources with // and /* */
    comments, trailing blanks and empty lines removed, so that a comment
    edit leaves it (and the counter summary taken on that code) unchanged."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in TRAFFIC_SETS[which][1]:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = re.sub(r"//.*", "", line).rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def read_traffic_summary(kernel: str, which: str = "fpsa"):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when the summary is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_SETS[which][0])
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("traffic ") or line.startswith("kernel_source_sha256 "):
                parts = line.split()
                vals[parts[1] if parts[0] == "traffic" else parts[0]] = parts[-1]
    if vals.get("kernel_source_sha256") != kernel_source_hash(which):
        return None
    v = vals.get(kernel)
    return float(v) if v is not None else None


def algorithmic_bytes_per_iteration(K, N, L1, P, fused_source=True):
    """Bytes each kernel must move per FPSA iteration (FP64), by kernel name,
    with the number of launches of that kernel per iteration.  The workload's
    sweeps carry the scattering source and the moments (fused path), and,
    the slab having one cell type, its correction's Fokker-Planck source is
    formed inside fp_matvec (fused_source; otherwise by a gemm_f64_mfma
    launch).

    sweep_aggregate  phi and the external source in, the source q out (the
                     tile scan itself works on the tile in LDS)
    sweep_apply      q in, the half-step moments out
    gemm_fp_source   gemm_f64_mfma forming the Fokker-Planck source:
                     phi_half, phi_old in, s out
    gemm_fp_update   gemm_f64_mfma forming the corrected moments: phi_half,
                     phi_old and the interface inflow in, phi_new out
    fp_matvec        per cell Hm and Hb, the source vector (fused: phi_half
                     and phi_old instead), f and g written
    fp_chain         per cell G and Gb, f and g read, the local values written
    fp_carry         the chunk transfer products (P(P-1)/2 per direction)
    fp_fixup         per cell PsiF, PsiB, W, W rho and sig, the local values
                     read and the inflow written
    The small tables every block reads (E, Mt, Vt) come from cache and are
    not counted.
    """
    NH, b = N // 2, 8
    M2 = NH * NH
    out = {
        "sweep_aggregate": (b * (2 * K * L1 + 4 * K * N), 1),
        "sweep_apply": (b * (2 * K * N + 2 * K * L1), 1),
        "gemm_fp_update": (b * (6 * K * L1 + K * N), 1),
        "fp_chain": (K * b * (2 * M2 + 2 * N), 1),
        "fp_carry": (b * M2 * P * (P - 1), 1),
        "fp_fixup": (K * b * (5 * M2 + 2 * N), 1),
    }
    if fused_source:
        out["fp_matvec"] = (K * b * (2 * M2 + 4 * L1 + N), 1)
    else:
        out["gemm_fp_source"] = (b * (4 * K * L1 + K * N), 1)
        out["fp_matvec"] = (K * b * (2 * M2 + 2 * N), 1)
    return out


def copy_probe(mib: int) -> int:
    """Plain device-to-device copy of a known size, for calibrating the
    FETCH_SIZE / WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8}), flush=True)
    return 0


def _read_csv(directory: str, suffix: str):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _counter_per_dispatch(directory: str, counter: str):
    """[(kernel name, grid size, value in KiB)] per dispatch, in dispatch order."""
    rows = _read_csv(directory, "counter_collection.csv")
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        name, grid = r["Kernel_Name"], r.get("Grid_Size", "")
        prev = acc.get(key, (name, grid, 0.0))
        acc[key] = (name, grid, prev[2] + float(r["Counter_Value"]))
    return [acc[k] for k in sorted(acc)]


def summarize_profiles(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, header, which="fpsa"):
    """Print the traffic summary: per kernel the average HBM bytes per launch
    from the FETCH_SIZE and WRITE_SIZE passes, each scaled by the ratio of
    the plain copy's known size to what the same counter read for it."""
    def copy_kib(d, counter):
        disp = [x for x in _counter_per_dispatch(d, counter) if "copyBuffer" in x[0] or "copy" in x[0]]
        return max(x[2] for x in disp)
    f_copy = copy_kib(copy_fetch_dir, "FETCH_SIZE")
    w_copy = copy_kib(copy_write_dir, "WRITE_SIZE")
    f_fac = copy_bytes / 1024.0 / f_copy
    w_fac = copy_bytes / 1024.0 / w_copy
    fetch = _counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_per_dispatch(write_dir, "WRITE_SIZE")
    lines = [header.rstrip(), f"kernel_source_sha256 {kernel_source_hash(which)}",
             f"copy_probe bytes {copy_bytes} FETCH_KiB {f_copy:.1f} WRITE_KiB {w_copy:.1f} "
             f"fetch_factor {f_fac:.4f} write_factor {w_fac:.4f}"]
    for kid, sub in ROCPROF_NAME.items():
        if kid not in SET_KERNELS[which]:
            continue
        fv = [x[2] for x in fetch if sub in x[0]]
        wv = [x[2] for x in write if sub in x[0]]
        if not fv or not wv:
            continue
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        lines.append(f"traffic {kid} launches {len(fv)} FETCH_KiB_avg {fk:.1f} WRITE_KiB_avg {wk:.1f} "
                     f"bytes_per_launch {1024.0 * (fk * f_fac + wk * w_fac):.6g}")
    print("\n".join(lines))
    return 0


MFMA_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F64",
                 "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_BF16")
SIMDS = 1024  # 256 CUs x 4 SIMDs
XCDS = 8      # GRBM_GUI_ACTIVE comes back summed over the XCDs


def summarize_mfma(pmc_dir: str, stats_dir: str, header: str, kernels) -> int:
    """Per kernel (substring of its rocprofv3 name): MFMA busy share =
    SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x SIMDs), the active cycles
    being GRBM_GUI_ACTIVE / XCDs (rocprofv3 returns that counter summed over
    the 8 XCDs; rocprofv3's own MfmaUtil takes the per-XCD maximum), and the MFMA flops
    (MOPS x 512) per dispatch from one rocprofv3 --pmc pass, with the average
    duration of the same kernel from a --kernel-trace --stats run of the same
    command, so that the flops give a rate."""
    rows = _read_csv(pmc_dir, "counter_collection.csv")
    per = {}
    for r in rows:
        key = int(r["Dispatch_Id"])
        d = per.setdefault(key, {"name": r["Kernel_Name"]})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    stats = _read_csv(stats_dir, "kernel_stats.csv")
    lines = [header.rstrip()]
    for sub in kernels:
        ds = [d for d in per.values() if sub in d["name"]]
        st = [r for r in stats if sub in r["Name"]]
        if not ds:
            continue
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in ds) / len(ds)
        gui = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in ds) / len(ds)
        mops = {c: sum(d.get(f"SQ_INSTS_VALU_MFMA_MOPS_{c}", 0.0) for d in ds) / len(ds) for c in ("F64", "F32", "BF16")}
        flops = {c: 512.0 * v for c, v in mops.items()}
        avg_ns = (sum(float(r["TotalDurationNs"]) for r in st) / sum(int(r["Calls"]) for r in st)) if st else None
        rate = {c: (f / (avg_ns * 1e-9) / 1e12 if avg_ns else None) for c, f in flops.items() if f}
        lines.append(f"mfma {sub!r} dispatches {len(ds)} busy_pct {100.0 * busy / max(gui / XCDS * SIMDS, 1.0):.1f} "
                     f"flops_per_dispatch " + " ".join(f"{c}={f:.4g}" for c, f in flops.items() if f) +
                     (f" avg_ns {avg_ns:.0f} TFLOPs " + " ".join(f"{c}={v:.1f}" for c, v in rate.items())
                      if avg_ns else ""))
    print("\n".join(lines))
    return 0


def summarize_stats(stats_dir: str, header: str, top: int = 16) -> int:
    """The kernels of a rocprofv3 --kernel-trace --stats run with the largest
    total time, as its kernel_stats.csv rows."""
    rows = _read_csv(stats_dir, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    lines = [header.rstrip(), f"# Columns: {', '.join(cols)} (top {top} by total time)",
             ",".join(f'"{c}"' for c in cols)]
    for r in rows[:top]:
        lines.append(",".join(f'"{r[c]}"' if c == "Name" else r[c] for c in cols))
    print("\n".join(lines))
    return 0


def marginal_iteration(torch, S, q, phi, n_lo: int, n_hi: int):
    """Wall time of one more source iteration, from solves of n_lo and n_hi
    iterations (kernel timing off: the graph-replayed solve), and the solve's
    fixed cost (FP32 conversion of phi^0, selection of the final iterate,
    history read-backs) that the difference removes."""
    t = {}
    for n in (n_lo, n_hi):
        phi.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.solve("si", tol=0.0, max_iter=n, q_ext=q, phi=phi, history=False)
        torch.cuda.synchronize()
        t[n] = time.perf_counter() - t0
    per = (t[n_hi] - t[n_lo]) / (n_hi - n_lo)
    return per, t[n_lo] - n_lo * per


def batched_measurement(torch, snfpsa, sw, reps: int = 5, si_iters: int = 3) -> dict:
    """The 4096-slab batch: FP32 sweeps of every (slab, angle) in one launch,
    timed per launch with HIP events, against the HBM roofline (16 bytes per
    cell-angle: two FP32 nodal sources read, two nodal fluxes written); and
    a few batched source iterations (source GEMM + sweep + moments with the
    FP64 stopping test) in FP32 and with the split-BF16 source GEMM."""
    import numpy as np
    probs = sw.batched_slabs(4096, with_source=False)
    cells = sum(p.K for p in probs)
    ca = sum(p.K * p.N for p in probs)
    # slabs whose moments after the timed iterations are checked against
    # the oracle: the shortest of every N, the longest, the largest c
    Ks = np.array([p.K for p in probs])
    picks = {int(np.argmax(Ks)), int(np.argmax([p.meta["c"] for p in probs]))}
    for N in sorted({p.N for p in probs}):
        idx = [b for b, p in enumerate(probs) if p.N == N]
        picks.add(min(idx, key=lambda b: probs[b].K))
    picks = sorted(picks)
    offs = np.cumsum([0] + [p.K * 2 * (p.L + 1) for p in probs])
    samples = {"problems": {b: probs[b] for b in picks}, "iterations": si_iters}
    out = {"workload": ("batch4096: 4096 slabs, K ~ U[256,8192], N in {16,32,64,128}, L = N-1, "
                        "HG / screened-Rutherford, c ~ U[0.9,0.9999], 1-8 regions, q = 1, vacuum"),
           "cells": cells, "cell_angles": ca}
    # algorithmic bytes of one fused iteration: the FP32 iterate read by the
    # aggregate and apply passes and written once (24 (L+1) bytes per cell),
    # the isotropic source's two node values read by both passes (16 bytes)
    fused_bytes = float(sum(p.K * (24 * (p.L + 1) + 16) for p in probs))
    for prec in ("f32", "f32_unfused", "bf16x3"):
        S = snfpsa.SlabSolver(probs, fp_scheme="none", precision="f32" if prec == "f32_unfused" else prec)
        if prec == "f32_unfused":
            S.set_fused_iteration(False)
        q = torch.ones(S.psi_len, dtype=torch.float32, device="cuda")
        r = {"fused": S.fused_iteration()["enabled"]}
        if prec == "f32":
            out["sweep_autotune"] = S.sweep_tuning()
            psi = S.psi_tensor()
            S.sweep(q, psi)
            torch.cuda.synchronize()
            S.set_kernel_timing(True)
            t0 = time.perf_counter()
            for _ in range(reps):
                S.sweep(q, psi)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            kt = S.kernel_timing()
            S.set_kernel_timing(False)
            n, ms = kt["sweep_batch_f32"]
            t = ms / max(n, 1) * 1e-3
            gbs = 16.0 * ca / t / 1e9
            out["sweep_api_layout"] = {"kernel": "sweep_batch_f32 ([cell][node][angle] layout of sn_sweep)",
                                       "avg_launch_ms": t * 1e3, "wall_ms": wall * 1e3,
                                       "cell_angle_updates_per_s": ca / t, "achieved": gbs, "unit": "GB/s",
                                       "frac": gbs / HBM_PEAK_GBS}
            del psi
        phi = S.phi_tensor()
        phi.zero_()
        S.solve("si", tol=0.0, max_iter=1, q_ext=q, phi=phi, history=False)  # warm-up, graph capture
        per, fixed = marginal_iteration(torch, S, q, phi, 2, 2 + 2 * si_iters)
        phi.zero_()
        torch.cuda.synchronize()
        S.set_kernel_timing(True)
        S.solve("si", tol=0.0, max_iter=si_iters, q_ext=q, phi=phi, history=False)
        torch.cuda.synchronize()
        kt = S.kernel_timing()
        S.set_kernel_timing(False)
        ph = phi.cpu().numpy()
        samples[prec] = {b: ph[offs[b]:offs[b + 1]].copy() for b in picks}
        r["ms_per_iteration"] = per * 1e3
        r["solve_fixed_ms"] = fixed * 1e3
        r["cell_angle_updates_per_s"] = ca / per
        r["kernels_avg_ms"] = {k: v[1] / v[0] for k, v in kt.items() if v[0]}
        if r["fused"]:
            # fused passes: launches per iteration = classes (aggregate and
            # apply) + 1 (scan); their summed time against the byte model
            kt_ms = sum(kt[k][1] for k in ("fused_aggregate", "fused_scan", "fused_apply") if k in kt)
            t_it = kt_ms / si_iters * 1e-3
            gbs = fused_bytes / t_it / 1e9
            sp = "_sp" if prec == "bf16x3" else ""
            parts = [read_traffic_summary("fused_scan", "batch")] + [
                None if (v := read_traffic_summary(f"fused_{k}{sp}<{w}>", "batch")) is None else v * n
                for w, n in FUSED_LAUNCHES.items() for k in ("aggregate", "apply")]
            traffic = None if any(v is None for v in parts) else sum(parts)
            r["roofline"] = {"bound": "hbm", "kernels": "fused_aggregate + fused_scan + fused_apply",
                             "kernel_ms_per_iteration": t_it * 1e3, "algorithmic_bytes_per_iteration": fused_bytes,
                             "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                             "traffic_per_iteration": traffic}
        if prec == "f32_unfused":
            # the solve's sweep (direction-major workspace): the batched-sweep roofline
            n, ms = kt["sweep_batch_f32"]
            t = ms / max(n, 1) * 1e-3
            gbs = 16.0 * ca / t / 1e9
            out["sweep"] = {"kernel": "sweep_batch_dm", "bound": "hbm", "avg_launch_ms": t * 1e3,
                            "cell_angle_updates_per_s": ca / t, "bytes_per_cell_angle": 16,
                            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                            "traffic": read_traffic_summary("sweep_batch_dm", "batch"),
                            "algorithmic_bytes_per_launch": 16.0 * ca}
        out[f"si_{prec}"] = r
        del phi, q
        S.close()
        torch.cuda.empty_cache()
    return out, samples


def batched_fpsa_slice(torch, snfpsa, sw):
    """FP64 FPSA-WFD in batched launches on a 256-slab slice of the batch
    recipe with K in [256, 512] (per-cell Fokker-Planck factors; the full
    recipe's per-cell factors would not fit), q = 1, tol 1e-9: setup time,
    one timed solve after a warm-up, iteration counts.  Returns the report
    and, for the oracle check of the cpu_baseline leg, sampled slabs with
    their moments."""
    import numpy as np
    probs = sw.batched_slabs(256, seed=31, k_range=(256, 512))
    cells = sum(p.K for p in probs)
    ca = sum(p.K * p.N for p in probs)
    t0 = time.perf_counter()
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd")
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    q = torch.ones(S.psi_len, dtype=torch.float64, device="cuda")
    tol = 1e-9
    S.solve("fpsa", tol=tol, max_iter=500, q_ext=q, history=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = S.solve("fpsa", tol=tol, max_iter=500, q_ext=q, history=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    its = np.array(r["iters"])
    updates = float(sum(int(i) * p.K * p.N for i, p in zip(its, probs)))
    phi = r["phi"].cpu().numpy()
    offs = np.cumsum([0] + [p.K * 2 * (p.L + 1) for p in probs])
    picks = sorted({int(np.argmax([p.meta["c"] for p in probs])),
                    next(b for b, p in enumerate(probs) if p.N == 128)})
    samples = {"tol": tol, "slabs": {b: (probs[b], phi[offs[b]:offs[b + 1]].copy(), int(its[b])) for b in picks}}
    S.close()
    out = {"workload": ("batch slice: 256 slabs of the batch recipe with K ~ U[256,512], N in {16,32,64,128}, "
                        "L = N-1, c ~ U[0.9,0.9999], q = 1, vacuum; FP64 FPSA-WFD, per-cell factors, tol 1e-9"),
           "cells": cells, "cell_angles": ca, "setup_s": setup, "solve_ms": t * 1e3, "status": r["status"],
           "iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
           "cell_angle_updates_per_s": updates / t}
    return out, samples


def batched_fpsa_oracle_check(samples) -> dict:
    """The sampled slabs of the FPSA slice against the oracle's FPSA solve:
    iteration counts and moments relative to the slab's largest."""
    import numpy as np
    import oracle
    out = {}
    for b, (p, phi, it) in samples["slabs"].items():
        ref = oracle.solve(p, "fpsa", "wfd", tol=samples["tol"], max_iter=500)
        out[str(b)] = {"K": p.K, "N": p.N, "c": p.meta["c"], "iterations": it, "oracle_iterations": int(ref["iters"]),
                       "max_rel": float(np.abs(phi - ref["phi"].ravel()).max() / np.abs(ref["phi"]).max())}
    return out


def batched_oracle_check(samples) -> dict:
    """Moments of the sampled slabs after the timed source iterations (from
    zero, q = 1) against the same iterations of the FP64 oracle; relative to
    the slab's largest moment."""
    import numpy as np
    import oracle
    out = {"iterations": samples["iterations"], "slabs": {}}
    worst = {"f32": 0.0, "f32_unfused": 0.0, "bf16x3": 0.0}
    for b, p in samples["problems"].items():
        p.q = np.ones((p.K, 2, p.N))
        ref = oracle.solve(p, "si", tol=0.0, max_iter=samples["iterations"])["phi"].ravel()
        p.q = np.zeros(0)
        e = {prec: float(np.abs(samples[prec][b] - ref).max() / np.abs(ref).max()) for prec in worst}
        out["slabs"][str(b)] = {"K": p.K, "N": p.N, "c": p.meta["c"], "kernel": p.meta["kernel"], **e}
        for prec in worst:
            worst[prec] = max(worst[prec], e[prec])
    out.update({f"{prec}_max_rel": v for prec, v in worst.items()})
    return out


def precision_ladder(torch, snfpsa, sw, iters: int = 10):
    """The single large slab (2^20 cells, S_256, L = 255, SRK eta = 1e-6,
    c = 0.9999, 16 regions, q = 1): `iters` source iterations from phi^0 = 0
    and one scattering-source GEMM in FP64, FP32 and split-BF16, timed per
    kernel with HIP events, with the errors of the FP32 / split-BF16 results
    relative to the FP64 path.  Returns the report and, for the oracle check
    of the cpu_baseline leg, the sampled cells with their FP64 moments and
    every precision's scattering source there."""
    import numpy as np
    p = sw.large_slab()
    K, N, L1 = p.K, p.N, p.L + 1
    flops = 2.0 * 2 * K * N * L1
    out = {"workload": ("large slab: 2^20 cells, S_256, L = 255, screened Rutherford eta = 1e-6, c = 0.9999, "
                        "16 regions, q = 1, vacuum"), "cells": K, "angles": N, "L": L1 - 1, "si_iterations": iters,
           "scatter_gemm_flop": flops}
    # sampled cells: both boundary layers, both sides of every region
    # interface, and random interior cells
    rng = np.random.Generator(np.random.PCG64(7))
    edges = np.flatnonzero(np.diff(p.sigma_t)) if np.ndim(p.sigma_t) else np.zeros(0, int)
    cells = np.unique(np.concatenate([np.arange(8), K - 1 - np.arange(8), edges, edges + 1,
                                      rng.choice(K, size=48, replace=False)]))
    samples = {"problem": p, "cells": cells}
    f64 = {}
    for prec in ("f64", "f32", "bf16x3"):
        S = snfpsa.SlabSolver([p], fp_scheme="none", precision=prec)
        scan = S.scan_tuning() if prec != "f64" else None
        q = torch.ones(S.psi_len, dtype=S.qdtype, device="cuda")
        phi = S.phi_tensor()
        phi.zero_()
        S.solve("si", tol=0.0, max_iter=1, q_ext=q, phi=phi, history=False)  # warm-up, graph capture
        per, fixed = marginal_iteration(torch, S, q, phi, 2, 6)
        phi.zero_()
        torch.cuda.synchronize()
        S.set_kernel_timing(True)
        S.solve("si", tol=0.0, max_iter=iters, q_ext=q, phi=phi, history=False)
        torch.cuda.synchronize()
        kt = S.kernel_timing()
        S.set_kernel_timing(False)
        r = {"ms_per_iteration": per * 1e3, "solve_fixed_ms": fixed * 1e3,
             "kernels_avg_ms": {k: v[1] / v[0] for k, v in kt.items() if v[0]}}
        if scan is not None:
            r["scan_autotune"] = scan
        phi_h = phi.cpu().numpy()
        # the scattering source of the FP64 path's final moments, timed alone
        src_in = f64["phi"] if prec != "f64" else phi
        qo = S.psi_tensor()
        S.scatter_source(src_in, None, qo)
        torch.cuda.synchronize()
        S.set_kernel_timing(True)
        S.scatter_source(src_in, None, qo)
        torch.cuda.synchronize()
        kt = S.kernel_timing()
        S.set_kernel_timing(False)
        gk = "gemm_f64_mfma" if prec == "f64" else "src_batch"
        n, ms = kt[gk]
        t = ms / max(n, 1) * 1e-3
        # operands of the boundary call: FP64 moments in, sigma_s (FP64 for
        # the FP64 handle, FP32 per cell otherwise) and q out
        qb, sb = (8, 8) if prec == "f64" else (4, 4)
        nbytes = 8.0 * 2 * K * L1 + sb * K * L1 + qb * 2.0 * K * N
        gbs = nbytes / t / 1e9
        if prec == "bf16x3":
            # three BF16 products per FP32 one (~1.7e12 flop in 0.7 ms at
            # the dense BF16 peak) against 7.5 GB of FP32 / FP64 operands:
            # the split product is bound by HBM
            r["scatter_gemm"] = {"kernel": gk, "bound": "hbm", "ms": t * 1e3, "achieved": gbs,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                 "bytes": nbytes, "TFLOPs_fp32_equivalent": flops / t / 1e12}
        else:
            peak = {"f64": 78.6, "f32": 157.3}[prec]
            r["scatter_gemm"] = {"kernel": gk, "bound": "mfma", "ms": t * 1e3, "achieved": flops / t / 1e12,
                                 "peak": peak, "unit": "TFLOP/s", "frac": flops / t / 1e12 / peak,
                                 "hbm_GBs": gbs, "bytes": nbytes}
        q_h = qo.cpu().numpy().astype(np.float64)
        samples[prec] = q_h.reshape(K, 2, N)[cells].copy()
        if prec == "f64":
            f64 = {"phi": phi, "phi_h": phi_h, "q": q_h}
            samples["phi"] = phi_h.reshape(K, 2, L1)[cells].copy()
        else:
            r["phi_rel_err_vs_f64"] = float(np.abs(phi_h - f64["phi_h"]).max() / np.abs(f64["phi_h"]).max())
            r["scatter_rel_err_vs_f64"] = float(np.abs(q_h - f64["q"]).max() / np.abs(f64["q"]).max())
        out[prec] = r
        del q, qo, phi_h, q_h
        if prec != "f64":
            del phi
        S.close()
        torch.cuda.empty_cache()
    del f64
    torch.cuda.empty_cache()
    return out, samples


def differentiation_measurement(torch, snfpsa, sw, tol: float = 1e-11) -> dict:
    """256 slabs x 4096 cells, S_64 (L = 63), HG g = 0.95, per-cell
    sigma_t ~ U[0.5, 2] and c ~ U[0.95, 0.999], q = 1, vacuum: the gradient
    of every slab's exit current with respect to every cell's sigma_t and
    sigma_{s,l}.  One gradient evaluation = forward FPSA solve + adjoint FPSA
    solve (reflected forward problem) + regeneration sweeps and gradient
    kernels; slab-mean Fokker-Planck coefficients (shared factorisations)."""
    import numpy as np
    probs = sw.differentiation_batch(256, with_source=False)
    K, N = probs[0].K, probs[0].N
    cells = sum(p.K for p in probs)
    t0 = time.perf_counter()
    S = snfpsa.SlabSolver(probs, fp_scheme="wfd", fp_coefficients="mean")
    setup = time.perf_counter() - t0
    qe = torch.ones(S.psi_len, dtype=torch.float64, device="cuda")
    c = S.exit_current_weights()

    def gradient():
        r = S.solve("fpsa", tol=tol, max_iter=1000, q_ext=qe, history=False)
        a = S.solve_adjoint(c, "fpsa", tol=tol, max_iter=1000)
        J, gt, gs = S.response_gradient(r["phi"], c, a["phi_y"], q_ext=qe)
        return r, a, J, gt, gs

    gradient()
    torch.cuda.synchronize()
    S.set_kernel_timing(True)
    t0 = time.perf_counter()
    r, a, J, gt, gs = gradient()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = S.kernel_timing()
    S.set_kernel_timing(False)
    its = sum(r["iters"]) + sum(a["iters"])
    out = {"workload": ("differentiation batch: 256 slabs x 4096 cells, S_64, L = 63, HG g = 0.95, per-cell "
                        "sigma_t ~ U[0.5,2], c ~ U[0.95,0.999], q = 1, vacuum; exit-current gradients"),
           "cells": cells, "angles": N, "tol": tol, "setup_s": setup,
           "seconds_per_gradient": wall,
           "forward_iterations_mean": float(np.mean(r["iters"])),
           "adjoint_iterations_mean": float(np.mean(a["iters"])),
           "cell_angle_updates_per_s": its * K * N / wall,
           "gradient_entries": int(gt.numel() + gs.numel()),
           "kernels_ms": {k: v[1] for k, v in kt.items() if v[0]},
           "finite": bool(torch.isfinite(gt).all()) and bool(torch.isfinite(gs).all())}
    dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
    out["dominant_kernel"] = dom
    out["status"] = {"forward": r["status"], "adjoint": a["status"]}
    # error of sampled gradient entries against FP64 central differences of
    # the exit current: slab 17 re-solved alone (same slab-mean Fokker-Planck
    # coefficients), parameters sigma_t, c, g of cells near the exit face;
    # chain rule from dJ/dsigma_t, dJ/dsigma_{s,l} of the HG moments
    # sigma_{s,l} = c sigma_t g^l
    b = 17
    p = probs[b]
    L = p.L
    gt_b = gt[b * K:(b + 1) * K].cpu().numpy()
    gs_b = gs[b * K * (L + 1):(b + 1) * K * (L + 1)].cpu().numpy().reshape(K, L + 1)
    J_b = float(J[b])
    S.close()
    del qe, c, J, gt, gs
    torch.cuda.empty_cache()
    st0, c0, g0 = p.sigma_t.copy(), p.meta["c"].copy(), p.meta["g"].copy()
    lpow = np.arange(L + 1)

    def analytic(which, k):
        gl = g0[k] ** lpow
        if which == "sigma_t":
            return gt_b[k] + float(np.dot(gs_b[k], c0[k] * gl))
        if which == "c":
            return float(np.dot(gs_b[k], st0[k] * gl))
        return float(np.dot(gs_b[k][1:], c0[k] * st0[k] * lpow[1:] * g0[k] ** (lpow[1:] - 1)))

    S1 = snfpsa.SlabSolver([p], fp_scheme="wfd", fp_coefficients="mean")
    q1 = torch.ones(S1.psi_len, dtype=torch.float64, device="cuda")
    pe = torch.zeros(S1.exit_len, dtype=torch.float64, device="cuda")

    def exit_current(st, cc, gg):
        S1.update_cross_sections(st, (cc * st)[:, None] * gg[:, None] ** lpow[None, :])
        rr = S1.solve("fpsa", tol=tol, max_iter=1000, q_ext=q1, psi_exit=pe, history=False)
        assert rr["status"] == 0
        return float(S1.exit_current(pe)[0])

    rng = np.random.Generator(np.random.PCG64(6))
    errs = []
    for i in range(8):
        which = ("sigma_t", "c", "g")[i % 3]
        k = int(K - 1 - rng.integers(0, 200))
        v = {"sigma_t": st0, "c": c0, "g": g0}
        d = 1e-5 * v[which][k]
        vals = []
        for sgn in (1.0, -1.0):
            w = {n: a.copy() for n, a in v.items()}
            w[which][k] += sgn * d
            vals.append(exit_current(w["sigma_t"], w["c"], w["g"]))
        fd = (vals[0] - vals[1]) / (2 * d)
        errs.append((which, k, fd, analytic(which, k)))
    J1 = exit_current(st0, c0, g0)
    S1.close()
    del q1, pe
    torch.cuda.empty_cache()
    fds = np.array([e[2] for e in errs])
    floor = 1e-3 * np.abs(fds).max()
    rel_errs = [abs(e[2] - e[3]) / max(abs(e[2]), floor) for e in errs]
    out["error_vs_finite_differences"] = {
        "slab": b, "samples": len(errs), "max_rel": float(max(rel_errs)),
        "entries": [{"param": e[0], "cell": e[1], "fd": e[2], "adjoint": e[3]} for e in errs],
        "J_batch": J_b, "J_single_slab": J1}
    return out, {"problem": p, "J": J_b}


def differentiation_oracle_check(sample) -> dict:
    """Exit current of the sampled slab of the gradient batch against the
    FP64 oracle's FPSA solution of the same slab (the gradient's value)."""
    import numpy as np
    import oracle
    p = sample["problem"]
    p.q = np.ones((p.K, 2, p.N))
    t0 = time.perf_counter()
    r = oracle.solve(p, "fpsa", "wfd", tol=1e-12, max_iter=500)
    t = time.perf_counter() - t0
    Jref = float((oracle.exit_current_weights(p.K, p.N) * r["psi"]).sum())
    return {"J_gpu": sample["J"], "J_oracle": Jref, "rel_err": abs(sample["J"] - Jref) / abs(Jref),
            "oracle_seconds": t}


def precision_converged(torch, snfpsa, sw) -> dict:
    """Converged low-precision solves at the 4096-slab recipe's high
    scattering ratios: four slabs (K 256-384, N 16 / 32 / 64, c from 0.99 to
    0.9999), FP32 source iteration run to its floor and FP32 / split-BF16
    source iterations refined by FP64 residuals, each against the FP64
    oracle's fixed point."""
    import numpy as np
    import oracle
    pool = sw.batched_slabs(40, seed=23, k_range=(256, 384))
    probs = []
    for N, c in ((16, 0.99), (32, 0.999), (64, 0.9999), (16, 0.9999)):
        p = next(x for x in pool if x.N == N and x not in probs)
        p.sigma_s = p.sigma_s * (c / p.meta["c"])
        p.meta["c"] = c
        probs.append(p)
    t0 = time.perf_counter()
    refs = []
    for p in probs:
        # to 1e-13 of the slab's largest moment: FPSA to 1e-8, then on from there
        r1 = oracle.solve(p, "fpsa", "wfd", tol=1e-8, max_iter=1000)
        sc = float(np.abs(r1["phi"]).max())
        refs.append(oracle.solve(p, "fpsa", "wfd", tol=1e-13 * sc, max_iter=1000, phi0=r1["phi"])["phi"].ravel())
    t_oracle = time.perf_counter() - t0
    scale = max(float(np.abs(r).max()) for r in refs)
    offs = np.cumsum([0] + [p.K * 2 * (p.L + 1) for p in probs])

    def errs(phi):
        return [float(np.abs(phi[offs[i]:offs[i + 1]] - r).max() / np.abs(r).max()) for i, r in enumerate(refs)]

    qe = torch.from_numpy(np.concatenate([p.q.ravel() for p in probs]))
    out = {"slabs": [{"K": p.K, "N": p.N, "c": p.meta["c"], "kernel": p.meta["kernel"]} for p in probs],
           "oracle_seconds": t_oracle}
    # FP32 source iteration to its floor, each slab on its own handle with a
    # stopping test at 64 eps32 of its own largest moment
    eps32 = float(np.finfo(np.float32).eps)
    f32 = {"iters": [], "status": [], "seconds": 0.0, "rel_err": []}
    for i, p in enumerate(probs):
        S = snfpsa.SlabSolver([p], fp_scheme="none", precision="f32")
        t0 = time.perf_counter()
        r = S.solve("si", tol=64 * eps32 * float(np.abs(refs[i]).max()), max_iter=60000,
                    q_ext=torch.from_numpy(p.q.ravel()).float().cuda(), history=False)
        torch.cuda.synchronize()
        f32["seconds"] += time.perf_counter() - t0
        f32["iters"].append(r["iters"][0])
        f32["status"].append(r["status"])
        f32["rel_err"].append(float(np.abs(r["phi"].cpu().numpy() - refs[i]).max() / np.abs(refs[i]).max()))
        S.close()
    out["f32_si"] = f32
    hi = snfpsa.SlabSolver(probs, fp_scheme="none")
    for prec in ("f32", "bf16x3"):
        lo = snfpsa.SlabSolver(probs, fp_scheme="none", precision=prec)
        t0 = time.perf_counter()
        rr = snfpsa.solve_refined(lo, hi, q_ext=qe.cuda(), tol=1e-12 * scale, tol_lo=1e-5 * scale, inner_rel=1e-2,
                                  max_steps=12, max_iter=60000)
        torch.cuda.synchronize()
        out[f"{prec}_refined"] = {"steps": rr["steps"], "status": rr["status"], "inner_iters": rr["inner_iters"],
                                  "seconds": time.perf_counter() - t0, "rel_err": errs(rr["phi"].cpu().numpy())}
        lo.close()
    hi.close()
    torch.cuda.empty_cache()
    return out


def ladder_oracle_check(samples) -> dict:
    """Scattering source of every precision at the sampled cells against the
    FP64 oracle evaluated on the same FP64 moments."""
    import numpy as np
    import oracle
    p, cells = samples["problem"], samples["cells"]
    t0 = time.perf_counter()
    ref = oracle.scatter_source(samples["phi"], p.sigma_s[cells], p.N)
    t = time.perf_counter() - t0
    scale = np.abs(ref).max()
    return {"cells": int(len(cells)), "oracle_seconds": t,
            **{f"{prec}_max_rel": float(np.abs(samples[prec] - ref).max() / scale)
               for prec in ("f64", "f32", "bf16x3")}}


def progress(msg: str) -> None:
    """One line on stderr as a section of the run ends."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scheme", default="wfd", choices=["wfd", "mpd"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-runs", action="store_true",
                    help="skip the source-iteration and other-scheme solves")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 4096-slab batched FP32 sweep / source-iteration measurement")
    ap.add_argument("--no-ladder", action="store_true",
                    help="skip the large-slab FP64 / FP32 / split-BF16 precision ladder")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the 256-slab exit-current gradient measurement")
    ap.add_argument("--only", choices=("batch", "ladder", "diff"),
                    help="run only that configuration's section and print it (profiling)")
    ap.add_argument("--exact-iters", type=int, nargs="?", const=-1, default=None,
                    help="time solves that run exactly this many iterations (tol 0; without a value: "
                         "the converged count), so that no queued iteration is a no-op (profiling)")
    ap.add_argument("--copy-probe", type=int, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--summarize", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                      "COPY_WRITE_DIR", "COPY_BYTES"),
                    help="print the traffic summary from rocprofv3 --pmc output directories")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("PMC_DIR", "STATS_DIR"),
                    help="print the MFMA-activity summary from a rocprofv3 --pmc output directory and a "
                         "--kernel-trace --stats one of the same command")
    ap.add_argument("--mfma-kernels", nargs="*", default=["gemm_f64_tall", "src_batch_p<128", "mom_batch_p<128>",
                                                           "src_batch_p<256", "src_batch_sp<256", "mom_batch<256>"])
    ap.add_argument("--summarize-stats", metavar="STATS_DIR",
                    help="print the top kernels of a rocprofv3 --kernel-trace --stats output directory")
    ap.add_argument("--summary-top", type=int, default=16, help="kernels listed by --summarize-stats")
    ap.add_argument("--summary-header", default="# traffic summary")
    ap.add_argument("--summary-set", default="fpsa", choices=sorted(TRAFFIC_SETS),
                    help="kernel sources whose hash the summary records")
    args = ap.parse_args()
    if args.summarize_stats:
        return summarize_stats(args.summarize_stats, args.summary_header, args.summary_top)
    if args.summarize_mfma:
        return summarize_mfma(*args.summarize_mfma, args.summary_header, args.mfma_kernels)
    if args.summarize:
        fd, wd, cfd, cwd, cb = args.summarize
        return summarize_profiles(fd, wd, cfd, cwd, int(cb), args.summary_header, args.summary_set)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (independent slabs would shard "
              "across GPUs with no exchange but an all-reduce of the stopping flags).", file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe)

    import numpy as np
    import torch

    import paper_1907_13013_amd as snfpsa
    import sn_workloads as sw

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.only:
        # one configuration's section alone (profiling runs)
        snfpsa.load_library()
        fn = {"batch": lambda t, m, w: batched_measurement(t, m, w)[0],
              "diff": lambda t, m, w: differentiation_measurement(t, m, w)[0],
              "ladder": lambda t, m, w: precision_ladder(t, m, w)[0]}[args.only]
        print(json.dumps({args.only: fn(torch, snfpsa, sw)}), flush=True)
        return 0
    prob = sw.srk_slab_2000()
    K, N, L1 = prob.K, prob.N, prob.L + 1
    tol = 1e-8
    max_iter = 20000
    q = torch.from_numpy(prob.q.ravel().copy()).cuda()

    S = snfpsa.SlabSolver([prob], fp_scheme=args.scheme)
    phi = S.phi_tensor()

    def step(solver, method, exact=None):
        phi.zero_()
        if exact:
            return solver.solve(method, tol=0.0, max_iter=exact, q_ext=q, phi=phi, history=False)
        return solver.solve(method, tol=tol, max_iter=max_iter, q_ext=q, phi=phi, history=False)

    exact = args.exact_iters
    if exact is not None and exact <= 0:
        exact = step(S, "fpsa")["iters"][0]
    for _ in range(args.warmup):
        step(S, "fpsa", exact)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        r = step(S, "fpsa", exact)
        iters.append(r["iters"][0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    progress(f"timed FPSA steps: {ms_per_step:.3f} ms per solve")
    it = iters[-1]
    value = it * K * N / (ms_per_step * 1e-3)
    phi_gpu = phi.cpu().numpy().copy()

    out = {
        "metric": METRIC, "value": value, "unit": "cell-angle updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "srk_slab_2000", "cells": K, "angles": N, "L": L1 - 1,
                   "kernel": "screened Rutherford eta=1e-5", "c": 0.999, "source": 1.0,
                   "boundaries": "vacuum", "tol": tol, "method": f"fpsa-{args.scheme}"},
        "fpsa_iterations": it,
        "sweep_tiles": S.sweep_tuning(),
    }
    if exact:
        out["exact_iters"] = exact

    if not args.no_side_runs:
        # source iteration on the same problem (one warm-up, one timed solve)
        step(S, "si")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = step(S, "si")
        torch.cuda.synchronize()
        t_si = (time.perf_counter() - t0) * 1e3
        other = "mpd" if args.scheme == "wfd" else "wfd"
        S2 = snfpsa.SlabSolver([prob], fp_scheme=other)
        step(S2, "fpsa")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ro = step(S2, "fpsa")
        torch.cuda.synchronize()
        t_o = (time.perf_counter() - t0) * 1e3
        S2.close()
        out["si"] = {"iterations": rs["iters"][0], "ms": t_si,
                     "cell_angle_updates_per_s": rs["iters"][0] * K * N / (t_si * 1e-3)}
        out[f"fpsa_{other}"] = {"iterations": ro["iters"][0], "ms": t_o}
        out["speedup_fpsa_vs_si"] = t_si / ms_per_step
        # FPSA-preconditioned GMRES(30) on the same problem and tolerance
        step(S, "fpsa_gmres")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rg = step(S, "fpsa_gmres")
        torch.cuda.synchronize()
        t_g = (time.perf_counter() - t0) * 1e3
        out["fpsa_gmres"] = {"sweeps": rg["iters"][0], "ms": t_g, "status": rg["status"]}
        progress("side runs (SI, other scheme, FPSA-GMRES) done")

    # live per-kernel HIP-event timing over the same FPSA steps, replayed for
    # exactly the converged iteration count so that no queued iteration is a
    # no-op launch
    S.set_kernel_timing(True)
    for _ in range(args.steps):
        step(S, "fpsa", it)
    torch.cuda.synchronize()
    kt = S.kernel_timing()
    S.set_kernel_timing(False)
    fused_src = not kt.get("gemm_fp_source", (0, 0.0))[0]
    per_iter = algorithmic_bytes_per_iteration(K, N, L1, S.slab_info(0)["nchunks"], fused_src)
    # every kernel of the iteration against the HBM roofline, each GEMM
    # instance on its own; the dominant one (largest total time) is the line's
    # roofline
    kernels = {}
    for name, (launches, total_ms) in kt.items():
        if not launches or name not in per_iter:
            continue
        bytes_iter, launches_iter = per_iter[name]
        per_launch = bytes_iter / launches_iter
        avg_ms = total_ms / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        kernels[name] = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic_summary(name),
                         "avg_launch_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": per_launch,
                         "total_ms": total_ms}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"]) if kernels else None
    out["roofline"] = kernels.get(dom)
    out["roofline_per_kernel"] = {k: {"frac": v["frac"], "achieved": v["achieved"], "avg_launch_us": v["avg_launch_us"],
                                      "traffic": v["traffic"]} for k, v in kernels.items()}
    out["kernel_time_share"] = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1),
                                    "ms": v[1]} for k, v in kt.items() if v[0]}
    S.close()

    if not args.no_batch:
        out["batched"], batch_samples = batched_measurement(torch, snfpsa, sw)
        out["batched"]["fpsa_f64_slice"], fpsa_slice_samples = batched_fpsa_slice(torch, snfpsa, sw)
        progress("batched section done")
    if not args.no_ladder:
        out["precision_ladder"], ladder_samples = precision_ladder(torch, snfpsa, sw)
        progress("precision ladder done")
    if not args.no_diff:
        out["differentiation"], diff_sample = differentiation_measurement(torch, snfpsa, sw)
        progress("differentiation done")

    if not args.no_cpu_baseline:
        import oracle
        # the FP64 oracle on the host cores, timed like the paper's Sec. 4:
        # wall clock of the iterations only, the Fokker-Planck factorisation
        # being setup (reported beside it); FPSA to the full 1e-8 test, source
        # iteration on a bounded sample of iterations, each at one thread and
        # at all threads the box gives this process
        threads_all = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        si_sample = 100
        legs = {}
        ro = None
        for th in sorted({1, threads_all}):
            oracle.set_threads(th)
            used = oracle.get_threads()
            r_f = oracle.solve(prob, "fpsa", args.scheme, tol=tol, max_iter=max_iter)
            f_fac, f_it = oracle.last_timing()
            oracle.solve(prob, "si", tol=0.0, max_iter=si_sample)
            _, s_it = oracle.last_timing()
            legs[used] = {"fpsa_iterations": r_f["iters"], "fpsa_iterate_s": f_it, "fpsa_factor_s": f_fac,
                          "si_sample_iterations": si_sample, "si_s_per_iteration": s_it / si_sample}
            progress(f"oracle at {used} threads done")
            ro = r_f
        oracle.set_threads(threads_all)
        top = max(legs)
        si_iters = out["si"]["iterations"] if "si" in out else None
        for leg in legs.values():
            if si_iters:
                leg["si_extrapolated_s"] = leg["si_s_per_iteration"] * si_iters
                leg["cpu_speedup_fpsa_vs_si"] = leg["si_extrapolated_s"] / leg["fpsa_iterate_s"]
        out["cpu_baseline"] = {
            "value": legs[top]["fpsa_iterations"] * K * N / legs[top]["fpsa_iterate_s"],
            "unit": "cell-angle updates/s", "cores": top, "kind": "oracle",
            "sample": (f"srk_slab_2000 by the FP64 C oracle: one FPSA-{args.scheme} solve to 1e-8 "
                       f"({legs[top]['fpsa_iterations']} iterations, value = their updates / the iteration wall "
                       f"time, the one-time block-LU factorisation excluded as in the paper's timings) and "
                       f"{si_sample} source iterations extrapolated to the GPU's SI count; at 1 and {top} "
                       f"OpenMP threads"),
            "seconds": legs[top]["fpsa_iterate_s"], "by_threads": {str(k): v for k, v in legs.items()}}
        if not exact:
            ref = np.asarray(ro["phi"]).ravel()
            out["error_vs_oracle"] = {
                "max_abs": float(np.abs(phi_gpu.ravel() - ref).max()),
                "max_rel": float(np.abs(phi_gpu.ravel() - ref).max() / np.abs(ref).max()),
                "oracle_iterations": int(ro["iters"])}
        if not args.no_batch:
            out["batched"]["error_vs_oracle_sampled"] = batched_oracle_check(batch_samples)
            out["batched"]["fpsa_f64_slice"]["error_vs_oracle_sampled"] = batched_fpsa_oracle_check(fpsa_slice_samples)
            progress("batched oracle check done")
            out["batched"]["converged_high_c"] = precision_converged(torch, snfpsa, sw)
            progress("converged high-c precision check done")
        if not args.no_ladder:
            out["precision_ladder"]["scatter_vs_oracle_sampled"] = ladder_oracle_check(ladder_samples)
        if not args.no_diff:
            out["differentiation"]["exit_current_vs_oracle"] = differentiation_oracle_check(diff_sample)
            progress("differentiation oracle check done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
