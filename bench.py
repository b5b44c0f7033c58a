#!/usr/bin/env python
"""Benchmark of the log-polar self-gravity hot path on one MI355X.

Headline: cells/s of the forward map (F_r + F_phi) on the single-disk
1024 x 2048 log-polar workload (r in [0.01, 100], exponential disk with a 20%
m = 2 logarithmic spiral), FP32 FFT/multiply with FP64-built kernel spectra.
One step = one pf_forces call on that grid with the density already resident
in HBM.  Also reported: the FP64 path, the transpose (backward) in both
precisions, the 64-disk batched launch, the paper's polar case 1 as a patch
plan (source annulus and origin wedges on a 1024 x 1024 destination), the
Cartesian second-order method on a 1024 x 1024 grid, the one-time table
builds, the roofline of the dominant
kernel (the fused column pass) and the FP64 CPU oracle timed on the host's
cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-batched] [--forward-only [--transpose]] [--copy-reference]
                       [--cartesian N] [--batched-only]
--forward-only runs only the FP32 forward (headline, pass times, roofline),
for profiler runs, and with --transpose the FP32 transpose of the same plan
as well; --copy-reference adds five 64 MiB device-to-device copies
at the end, the known-size reference that calibrates the FETCH_SIZE and
WRITE_SIZE counters; --cartesian N and --batched-only time only the
Cartesian N x N plans or only the 64-disk batch (profiler runs).  Prints one
JSON line on stdout.
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

METRIC = "cells/s for F_r+F_phi at 1024x2048 (FP32 vs FP64, same GPU); backward cells/s"
N_R, N_PHI, R_MIN, R_MAX = 1024, 2048, 0.01, 100.0
HBM_PEAK_GBS = 8000.0


# Counter summary of the dominant kernel (FETCH_SIZE / WRITE_SIZE per
# dispatch with their copy-kernel calibration) and the sources it depends on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_cols_fwd_pf_f32_1024x2048_traffic.txt")
# Kernel-trace summary of the same kernel (mean launch duration under the
# profiler), for the cross-check of the event-timed roofline fraction.
TRACE_FILE = os.path.join(ROOT, "profiles", "k_cols_fwd_pf_f32_1024x2048_kernel_trace.md")
KERNEL_SOURCES = ("paper_1509_01450_amd/csrc/fft_core.hpp",
                  "paper_1509_01450_amd/csrc/pass_bodies.hpp",
                  "paper_1509_01450_amd/csrc/pf_passes.hip")


def kernel_source_hash():
    """Hash of the dominant kernel's sources with comments and white space
    removed (a comment edit does not change the kernel)."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(cols_shape):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel sources or its launch shape differ from
    those the counters were taken with."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for line in lines:
        if ":" in line and not line.startswith(("#", " ", "|")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv["source_hash"] != kernel_source_hash():
            return None
        if [int(x) for x in kv["cols_E_G"].split(",")] != list(cols_shape):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def profiled_mean_us(path, cols_shape):
    """Mean duration (us) of the dominant kernel in a committed kernel-trace
    summary, or None when its kernel sources or launch shape differ."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("|", " ", "#")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_hash") != kernel_source_hash():
            return None
        if [int(x) for x in kv.get("cols_E_G", "").split(",")] != list(cols_shape):
            return None
        return float(kv["avg_us"])
    except (OSError, KeyError, ValueError):
        return None


def cold_ms(torch, fn, n=20, flush_bytes=512 << 20):
    """Mean duration of one call with the caches cold: before each call a
    512 MiB buffer is written (twice the 256 MB last-level cache) on the same
    stream, outside the events that bracket the call."""
    scratch = torch.empty(flush_bytes // 4, dtype=torch.float32, device="cuda:0")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    fn()
    for i, (e0, e1) in enumerate(ev):
        scratch.fill_(float(i))
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    del scratch
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) / n


def copy_GBs(torch, nbytes, reps=20):
    """Device-to-device copy bandwidth (bytes read + written per second)."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_model():
    """CPU model name and the number of physical cores of the host."""
    name, cores = "unknown", set()
    try:
        with open("/proc/cpuinfo") as fh:
            phys = core = None
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name":
                    name = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    return name, (len(cores) or os.cpu_count())


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def path_bytes(n_r, n_phi, L, w):
    """Algorithmic HBM bytes of one forward call (three passes), with
    H = P/2 columns of the packed half spectrum:
    pass A reads sigma (R P w) and writes S (R H 2w); pass B reads S and the
    four half spectra (4 (L/2+1) H 2w) and writes Zr, Zp (2 R H 2w); pass C
    reads Zr, Zp and writes F_r, F_phi (2 R P w)."""
    H = n_phi // 2
    a = n_r * n_phi * w + n_r * H * 2 * w
    b = n_r * H * 2 * w + 4 * (L // 2 + 1) * H * 2 * w + 2 * n_r * H * 2 * w
    c = 2 * n_r * H * 2 * w + 2 * n_r * n_phi * w
    return a, b, c


def cart_path_bytes(n_x, n_y, Lx, Ly, w):
    """Algorithmic HBM bytes of one Cartesian forward call, H = L_y/2:
    pass A reads sigma (N_x N_y w) and writes the (S, Dy) pairs
    (N_x H 4w); pass B reads them, the six half spectra
    (2 H (L_x/2+1) (4w + 2w)) and writes the (Zx, Zy) pairs (N_x H 4w);
    pass C reads the pairs and writes F^x, F^y (2 N_x N_y w)."""
    H = Ly // 2
    a = n_x * n_y * w + n_x * H * 4 * w
    b = n_x * H * 4 * w + 2 * H * (Lx // 2 + 1) * 6 * w + n_x * H * 4 * w
    c = n_x * H * 4 * w + 2 * n_x * n_y * w
    return a, b, c


def time_calls(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per call


def median_call_ms(torch, fn, n=100):
    """Median over n calls of one call bracketed by its own HIP events
    (consecutive events on the launch stream; each interval holds one call
    and one event record)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    for _ in range(10):
        fn()
    ev[0].record()
    for i in range(n):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(n))
    return t[n // 2]


def sched(plan):
    s = plan.schedule()
    return {"rows1_E_G": list(s[0:2]), "rows2_E_G": list(s[2:4]), "cols_E_G": list(s[4:6]),
            "cols_adj_E_G": list(s[6:8])}


def time_graph(torch, fn, steps, warmup):
    """ms per step with the step captured once in a HIP graph (through
    torch.cuda.CUDAGraph on the current stream) and replayed `steps` times:
    the launch cost of a compiled caller, without the Python call path."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    ms = time_calls(torch, g.replay, steps, warmup)
    del g
    return ms


def pass_times(plan, a, b=None, backward=False, reps=100):
    """Mean duration (ms) of one launch of each pass, from HIP events on the
    launch stream around `reps` back-to-back launches of that pass."""
    plan.timed(a, b, backward, reps=5)
    return plan.timed(a, b, backward, reps=reps)


def cpu_baseline(sample_seconds=15.0):
    """The FP64 oracle's direct sums on a bounded random sample of output
    cells of the same 1024 x 2048 workload (tables built first, untimed)."""
    import numpy as np

    import oracle
    import workloads
    g = oracle.Grid(N_R, N_PHI, R_MIN, R_MAX)
    T = oracle.tables(g, 19)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    rng = np.random.default_rng(7)
    # calibrate on a small sample, then size the timed sample
    probe = rng.choice(N_R * N_PHI, 64, replace=False)
    t0 = time.perf_counter()
    oracle.forward(g, T, sig, probe)
    rate = 64 / max(time.perf_counter() - t0, 1e-6)
    n = int(max(128, min(N_R * N_PHI, rate * sample_seconds)))
    idx = rng.choice(N_R * N_PHI, n, replace=False)
    t0 = time.perf_counter()
    oracle.forward(g, T, sig, idx)
    dt = time.perf_counter() - t0
    model, phys = cpu_model()
    # the 128 x 128 grid in full (tables untimed)
    g1 = oracle.Grid(128, 128, 0.1, 10.0)
    T1 = oracle.tables(g1, 19)
    s1 = workloads.single_disk_blobs(g1.r_centres, g1.phi_centres)
    t0 = time.perf_counter()
    oracle.forward(g1, T1, s1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "cells/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": model, "physical_cores": phys,
            "c1_128x128_full_grid": {"s": dt1, "cells_per_s": 128 * 128 / dt1},
            "sample": "%d random output cells of the 1024x2048 workload (FP64 direct "
                      "O((N_r N_phi)^2) sums, %.1f s)" % (n, dt)}


def batched_detail(pf, torch, np, workloads, dev, K):
    """The 64-disk FP32 batch: eager and graph-replayed call times, cells/s,
    path bytes and their fraction of the HBM peak."""
    log("batched: 64 disks")
    sizes = workloads.batch_sizes(64)
    plans, sig_b = [], []
    t0 = time.perf_counter()
    for d, (nr, nphi) in enumerate(sizes):
        pb = pf.Plan(nr, nphi, 0.01, 100.0, dtype="f32")
        r_b, _, _ = pb.geometry()
        ph_b = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
        plans.append(pb)
        sig_b.append(torch.tensor(workloads.multiarm_disk(r_b, ph_b, d), dtype=torch.float32,
                                  device=dev))
    torch.cuda.synchronize()
    build_b = time.perf_counter() - t0
    outs = [(torch.empty_like(s), torch.empty_like(s)) for s in sig_b]
    msb = time_calls(torch, lambda: pf.forces_batched(plans, sig_b, outs), max(K // 4, 10), 5)
    msg = time_graph(torch, lambda: pf.forces_batched(plans, sig_b, outs), max(K // 4, 10), 5)
    bcells = sum(nr * nphi for nr, nphi in sizes)
    # transform length along u: the power of two at or above 2 N_r
    bbytes = sum(sum(path_bytes(nr, nphi, 1 << (2 * nr - 1).bit_length(), 4))
                 for nr, nphi in sizes)
    batched = {"workload": "64 disks, N_r in {256..1024}, N_phi in {256..2048}, FP32",
               "cells": bcells, "ms_per_call": msb, "cells_per_s": bcells / (msb * 1e-3),
               "path_bytes": bbytes,
               "path_frac_of_hbm_peak": bbytes / (msb * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "graph_ms_per_call": msg, "graph_cells_per_s": bcells / (msg * 1e-3),
               "table_build_s": build_b}
    return batched


def cartesian_detail(pf, torch, np, dev, NC, K, W):
    """Cartesian NC x NC grid (second-order method, sigma_D2 disk), FP32 and
    FP64: call time and the three passes' times, bytes and rates."""
    log("cartesian %d x %d" % (NC, NC))
    cart = {}
    xc = (np.arange(NC) + 0.5) / NC - 0.5
    Xc, Yc = np.meshgrid(xc, xc, indexing="ij")
    sig_c = np.clip(1.0 - (Xc ** 2 + Yc ** 2) / 0.25 ** 2, 0.0, None) ** 1.5
    for dt in ("f32", "f64"):
        t0 = time.perf_counter()
        pc = pf.CartPlan(NC, NC, 1.0 / NC, 1.0 / NC, dtype=dt, method="second")
        torch.cuda.synchronize()
        bc = time.perf_counter() - t0
        sc = torch.tensor(sig_c, dtype=pc.torch_dtype, device=dev)
        oc = (torch.empty_like(sc), torch.empty_like(sc))
        msc = time_calls(torch, lambda: pc.forces(sc, oc), max(K // 2, 10), W)
        pmc = pc.timed(sc, reps=100)
        _, _, Lx, Ly = pc.geometry()
        bts = cart_path_bytes(NC, NC, Lx, Ly, 4 if dt == "f32" else 8)
        cart[dt] = {"ms_per_call": msc, "cells_per_s": NC * NC / (msc * 1e-3), "pass_ms": pmc,
                    "pass_bytes": list(bts),
                    "pass_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(bts, pmc)],
                    "pass_B_frac_of_hbm_peak": bts[1] / (pmc[1] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "table_build_s": bc}
        pc.close()
    cart["workload"] = ("Cartesian %d x %d cells on [-0.5, 0.5]^2, sigma_D2 disk "
                        "(alpha = 0.25), second-order method" % (NC, NC))
    return cart


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--forward-only", action="store_true")
    ap.add_argument("--transpose", action="store_true")
    ap.add_argument("--copy-reference", action="store_true")
    ap.add_argument("--cartesian", type=int, default=0, metavar="N",
                    help="time only the Cartesian N x N plans (profiling runs)")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the 64-disk batch (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the single-disk and batched paths run on "
              "one device (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1509_01450_amd as pf
    import workloads

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    if args.cartesian:
        print(json.dumps(cartesian_detail(pf, torch, np, dev, args.cartesian, K, W)))
        return 0
    if args.batched_only:
        print(json.dumps(batched_detail(pf, torch, np, workloads, dev, K)))
        return 0
    cells = N_R * N_PHI
    out = {"metric": METRIC, "unit": "cells/s", "n_gpus": 1, "steps": K, "warmup": W,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}

    # ---- FP32 forward (headline) ------------------------------------------
    t0 = time.perf_counter()
    p32 = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f32")
    torch.cuda.synchronize()
    build32 = time.perf_counter() - t0
    rc, _, _ = p32.geometry()
    phi = (np.arange(N_PHI) + 0.5) * (2 * np.pi / N_PHI)
    sig_np = workloads.spiral_disk(rc, phi)
    s32 = torch.tensor(sig_np, dtype=torch.float32, device=dev)
    fr32, fp32 = torch.empty_like(s32), torch.empty_like(s32)
    log("fp32 forward: warmup %d, steps %d" % (W, K))
    f32 = lambda: p32.forces(s32, (fr32, fp32))
    ms32 = time_calls(torch, f32, K, W)
    ms32_graph = time_graph(torch, f32, K, W)
    ms32_median = median_call_ms(torch, f32)
    passes32 = pass_times(p32, s32)
    ms32_cold = None
    if not args.forward_only:   # profiled runs: warm launches only
        log("fp32 forward, caches cold")
        ms32_cold = cold_ms(torch, f32)
    L = p32_L = 2 * N_R
    bA, bB, bC = path_bytes(N_R, N_PHI, p32_L, 4)
    achieved = bB / (passes32[1] * 1e-3) / 1e9
    prof_us = profiled_mean_us(TRACE_FILE, p32.schedule()[4:6])

    out["value"] = cells / (ms32 * 1e-3)
    out["ms_per_step"] = ms32
    out["config"] = {"workload": "single disk log-polar %dx%d, r in [%g, %g], exponential disk "
                                 "+ 20%% m=2 log spiral, forward F_r+F_phi" % (N_R, N_PHI, R_MIN, R_MAX),
                     "n_r": N_R, "n_phi": N_PHI, "L_u": L, "n_tpz": 19, "precision":
                     "FP32 FFT + spectral multiply, FP64-built kernel spectra"}
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": measured_traffic(p32.schedule()[4:6])}
    out["detail"] = {
        "dominant_kernel": "k_cols_fwd_pf (u-FFT + spectral MAC with spectral radial slope + "
                           "two inverse u-FFTs; radial spectra prefetched to LDS)",
        "dominant_kernel_source_hash": kernel_source_hash(),
        "step_timing": "K back-to-back pf_forces calls between events on the launch stream",
        "median_call_ms_fp32": ms32_median,
        "median_call_timing": "median over 100 calls of one call between consecutive events",
        "roofline_timing": "achieved = algorithmic bytes of one pass-B launch / its mean "
                           "duration from HIP events on the launch stream around 100 "
                           "back-to-back launches (warm caches)",
        "roofline_frac_rocprof": (bB / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS
                                  if prof_us else None),
        "roofline_rocprof_avg_us": prof_us,
        "cold_ms_per_step_fp32": ms32_cold,
        "cold_cells_per_s_fp32": cells / (ms32_cold * 1e-3) if ms32_cold else None,
        "cold_path_frac_of_hbm_peak_fp32": ((bA + bB + bC) / (ms32_cold * 1e-3) / 1e9 / HBM_PEAK_GBS
                                            if ms32_cold else None),
        "cold_flush": "512 MiB written on the stream before each timed call, outside its events",
        "path_frac_of_hbm_peak_fp32": (bA + bB + bC) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "pass_sum_ms_fp32": sum(passes32),
        "graph_ms_per_step_fp32": ms32_graph,
        "graph_cells_per_s_fp32": cells / (ms32_graph * 1e-3),
        "schedule_fp32": sched(p32),
        "pass_ms_fp32": passes32, "pass_bytes_fp32": [bA, bB, bC],
        "pass_GBs_fp32": [b / (t * 1e-3) / 1e9 for b, t in zip((bA, bB, bC), passes32)],
        "path_bytes_fp32": bA + bB + bC,
        "path_GBs_fp32": (bA + bB + bC) / (ms32 * 1e-3) / 1e9,
        "table_build_s": {"fp32": build32},
    }
    if args.forward_only:
        if args.transpose:
            log("fp32 transpose")
            gr32, gp32 = torch.randn_like(s32), torch.randn_like(s32)
            gs32 = torch.empty_like(s32)
            msb32 = time_calls(torch, lambda: p32.backward(gr32, gp32, gs32), K, W)
            passesb32 = pass_times(p32, gr32, gp32, backward=True)
            out["detail"]["backward"] = {"fp32_ms": msb32, "fp32_cells_per_s": cells / (msb32 * 1e-3),
                                         "fp32_pass_ms": passesb32}
        finish(torch, out, args)
        return 0

    # ---- FP64 forward -----------------------------------------------------
    t0 = time.perf_counter()
    p64 = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f64")
    torch.cuda.synchronize()
    build64 = time.perf_counter() - t0
    s64 = torch.tensor(sig_np, dtype=torch.float64, device=dev)
    fr64, fp64 = torch.empty_like(s64), torch.empty_like(s64)
    log("fp64 forward")
    ms64 = time_calls(torch, lambda: p64.forces(s64, (fr64, fp64)), max(K // 2, 10), W)
    passes64 = pass_times(p64, s64)
    cA, cB, cC = path_bytes(N_R, N_PHI, L, 8)

    # ---- backward ---------------------------------------------------------
    log("backward")
    gr32, gp32 = torch.randn_like(s32), torch.randn_like(s32)
    gs32 = torch.empty_like(s32)
    msb32 = time_calls(torch, lambda: p32.backward(gr32, gp32, gs32), max(K // 2, 10), W)
    gr64, gp64 = gr32.double(), gp32.double()
    gs64 = torch.empty_like(gr64)
    msb64 = time_calls(torch, lambda: p64.backward(gr64, gp64, gs64), max(K // 4, 10), W)
    passesb32 = pass_times(p32, gr32, gp32, backward=True)

    # ---- C1: 128 x 128 on [0.1, 10], FP64 (launch-bound; no roofline claim) ----
    log("128 x 128 fp64")
    c1 = pf.Plan(128, 128, 0.1, 10.0, dtype="f64")
    rc1, _, _ = c1.geometry()
    ph1 = (np.arange(128) + 0.5) * (2 * np.pi / 128)
    s1 = torch.tensor(workloads.single_disk_blobs(rc1, ph1), dtype=torch.float64, device=dev)
    o1 = (torch.empty_like(s1), torch.empty_like(s1))
    ms_c1 = time_calls(torch, lambda: c1.forces(s1, o1), K, W)
    c1.close()
    c1_detail = {"workload": "128 x 128, r in [0.1, 10], (1+r^2)^-3/2 + 8 blobs, FP64",
                 "ms_per_call": ms_c1, "cells_per_s": 128 * 128 / (ms_c1 * 1e-3)}

    # ---- five-point slopes (slope order 4), same workload ----------------------
    log("slope order 4")
    so4 = {}
    for dt, sg in (("fp32", s32), ("fp64", s64)):
        p4 = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f32" if dt == "fp32" else "f64",
                     slope_order=4)
        o4 = (torch.empty_like(sg), torch.empty_like(sg))
        ms4 = time_calls(torch, lambda: p4.forces(sg, o4), max(K // 4, 10), W)
        so4[dt] = {"ms_per_call": ms4, "cells_per_s": cells / (ms4 * 1e-3),
                   "pass_ms": pass_times(p4, sg), "schedule": sched(p4)}
        p4.close()

    # ---- an azimuthal count of three times a power of two --------------------
    log("1024 x 1536")
    three_p = {"workload": "1024 x 1536 (N_phi = 3 x 512), r in [0.01, 100], spiral disk"}
    for dt in ("fp32", "fp64"):
        p3 = pf.Plan(N_R, 1536, R_MIN, R_MAX, dtype="f32" if dt == "fp32" else "f64")
        r3, _, _ = p3.geometry()
        ph3 = (np.arange(1536) + 0.5) * (2 * np.pi / 1536)
        s3 = torch.tensor(workloads.spiral_disk(r3, ph3), dtype=p3.torch_dtype, device=dev)
        o3 = (torch.empty_like(s3), torch.empty_like(s3))
        ms3 = time_calls(torch, lambda: p3.forces(s3, o3), max(K // 4, 10), W)
        three_p[dt] = {"ms_per_call": ms3, "cells_per_s": N_R * 1536 / (ms3 * 1e-3),
                       "pass_ms": pass_times(p3, s3), "schedule": sched(p3)}
        p3.close()

    # ---- batched ------------------------------------------------------------
    batched = None
    if not args.no_batched:
        batched = batched_detail(pf, torch, np, workloads, dev, K)

    # ---- Cartesian grid (second-order method, sigma_D2 disk) -----------------
    cart = cartesian_detail(pf, torch, np, dev, 1024, K, W)

    # ---- patches: the paper's polar case 1 at N_d = 1024 ---------------------
    log("patches: polar case 1, 1024 x 1024 destination")
    ND = 1024
    beta_d = 100.0 ** (1.0 / ND)
    n_s = int(round(np.log(1e-2 / (1e-4 * 8.0 / ND)) / np.log(beta_d)))
    k = -n_s + np.arange(n_s)
    rc_s = 1e-2 * beta_d ** k * 0.5 * (1.0 + beta_d)
    rh = 0.5 * 1e-2 * beta_d ** (-n_s)
    sd2 = lambda r: np.clip(1.0 - (r / 0.006) ** 2, 0.0, None) ** 1.5
    patches = {"workload": "polar case 1: sigma_D2 (alpha = 0.006) in a %d-row source "
                           "annulus and the origin wedges, acting on the mass-free "
                           "1024 x 1024 destination [0.01, 1]" % n_s}
    for dt in ("f32", "f64"):
        t0 = time.perf_counter()
        pp = pf.PatchPlan(n_s, -n_s, ND, ND, 1e-2, 1.0, wedges=True, dtype=dt, method="sim")
        torch.cuda.synchronize()
        bp = time.perf_counter() - t0
        ss = torch.tensor(np.repeat(sd2(rc_s)[:, None], ND, axis=1), dtype=pp.torch_dtype,
                          device=dev)
        sw = torch.full((ND,), float(sd2(np.array([rh]))[0]), dtype=pp.torch_dtype, device=dev)
        op = (torch.empty((ND, ND), dtype=pp.torch_dtype, device=dev),
              torch.empty((ND, ND), dtype=pp.torch_dtype, device=dev))
        msp = time_calls(torch, lambda: pp.forces(ss, sw, op), max(K // 2, 10), W)
        # the transpose with the wedges: cotangents on the destination ->
        # gradients on the source annulus and the wedge densities
        gb = (torch.empty_like(ss), torch.empty_like(sw))
        msb = time_calls(torch, lambda: pp.backward(op[0], op[1], gb), max(K // 2, 10), W)
        patches[dt] = {"ms_per_call": msp, "destination_cells_per_s": ND * ND / (msp * 1e-3),
                       "transpose_ms_per_call": msb, "table_build_s": bp}
        pp.close()

    out["detail"].update({
        "patches": patches,
        "cartesian": cart,
        "schedule_fp64": sched(p64),
        "fp64": {"ms_per_call": ms64, "cells_per_s": cells / (ms64 * 1e-3),
                 "pass_ms": passes64,
                 "pass_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip((cA, cB, cC), passes64)],
                 "path_GBs": (cA + cB + cC) / (ms64 * 1e-3) / 1e9},
        "backward": {"fp32_ms": msb32, "fp32_cells_per_s": cells / (msb32 * 1e-3),
                     "fp64_ms": msb64, "fp64_cells_per_s": cells / (msb64 * 1e-3),
                     "fp32_pass_ms": passesb32},
        "batched": batched,
        "slope_order_4": so4,
        "c1_128x128_fp64": c1_detail,
        "n_phi_1536": three_p,
    })
    out["detail"]["table_build_s"]["fp64"] = build64
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    finish(torch, out, args)
    return 0


def finish(torch, out, args):
    # measured copy bandwidth beside the 8 TB/s peak: 64 MiB (fits the
    # last-level cache) and 1 GiB (does not); not in profiled runs
    if not args.forward_only:
        cp = {"64MiB": copy_GBs(torch, 64 << 20), "1GiB": copy_GBs(torch, 1 << 30, reps=5),
              "peak": HBM_PEAK_GBS}
        out["detail"]["copy_GBs"] = cp
        # the path and pass B against what a plain copy reaches on this machine
        out["detail"]["path_frac_of_copy_fp32"] = out["detail"]["path_GBs_fp32"] / cp["1GiB"]
        out["detail"]["pass_B_frac_of_copy_fp32"] = out["roofline"]["achieved"] / cp["1GiB"]
    if args.copy_reference:
        log("copy reference: 5 x 64 MiB device-to-device")
        x = torch.ones(16 * 1024 * 1024, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
