#!/usr/bin/env python3
"""Benchmark of the generalized 2D correlation hot path on one MI355X.

One step = one corr2d_homo call through the C ABI on the m=256 x n=16384
band workload (128 Lorentzian/Gaussian bands, amplitudes 1e-3..1e2, noise
1e-4; upper triangle stored, FP32 output): the FFT tables, the radix FFT
transform with the FP64 centring fused in (m = 256 is a power of two in
[128, 1024]) writing split-BF16 operands in the default time basis (the
centred spectra and Noda's N Yc as an FFT correlation), and the split-BF16
MFMA contraction with its epilogue (normalization and unscaling).  Inputs
are resident in HBM before timing.

Prints ONE JSON line: throughput in correlation entries/s (stored
(Phi, Psi) pairs), the roofline of the contraction kernel (timed alone with
HIP events on the call's stream through the library's timing hook), the
error against the FP64 oracle over the full matrices, the same measurements
for the plain FP32, FP64 and BF16 forms and the other workloads, and the
oracle timed on the host.

The oracle serves two purposes here, both outside every timed region: the
CPU baseline (with the oracle's time on every workload), and the reference
values behind each error figure (every entry of every output, computed in
row blocks).  Every timed call runs through the HIP library alone.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("correlation entries/s and MFMA TFLOP/s at stated error vs oracle; "
          "split vs plain")
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "split_bf16": 2500.0, "bf16": 2500.0,
               "f16": 2500.0, "fp8_e4m3": 5000.0, "split_f16": 2500.0}
HBM_GBPS = 8000.0


def rel_fro(g, o):
    return float(np.linalg.norm(g - o) / np.linalg.norm(o))


def upper_oracle(oracle, torch, S, dev, block=1024):
    """The oracle's homocorrelation (Noda's kernel and norm) over the upper
    triangle, computed in row blocks of the direct route, as packed FP64
    planes on `dev`; returns (phi, psi, seconds the oracle took)."""
    t0 = time.perf_counter()
    Y, _ = oracle.dynamic(S)
    secs = time.perf_counter() - t0
    m, n = Y.shape
    tot = n * (n + 1) // 2
    phi = torch.empty(tot, dtype=torch.float64, device=dev)
    psi = torch.empty(tot, dtype=torch.float64, device=dev)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        t0 = time.perf_counter()
        po, qo = oracle.corr_ht_block(Y, Y, r0, r1, r0, n)
        secs += time.perf_counter() - t0
        mask = np.triu(np.ones((r1 - r0, n - r0), dtype=bool))
        a, b = r0 * n - (r0 * (r0 - 1)) // 2, r1 * n - (r1 * (r1 - 1)) // 2
        phi[a:b] = torch.as_tensor(po[mask], device=dev)
        psi[a:b] = torch.as_tensor(qo[mask], device=dev)
        del po, qo, mask
    return phi, psi, secs


def packed_diag(torch, n, dev):
    i = torch.arange(n, device=dev, dtype=torch.int64)
    return i * n - (i * (i - 1)) // 2


def aligned_to_packed_index(torch, n, dev):
    """Positions, in an UPPER_ALIGNED plane, of the entries of the packed
    order: (i, j) at i N32 - 32 (16 q (q-1) + r q) + (j - 32 q), i = 32 q + r."""
    i = torch.arange(n, device=dev, dtype=torch.int64)
    lens = n - i
    rows = torch.repeat_interleave(i, lens)
    j = torch.arange(rows.numel(), device=dev, dtype=torch.int64) - (torch.cumsum(lens, 0) - lens)[rows] + rows
    n32 = (n + 31) // 32 * 32
    q, r = rows // 32, rows % 32
    return rows * n32 - 32 * (16 * q * (q - 1) + r * q) + (j - 32 * q)


def full_counts(torch, g, o, diag, chunk=1 << 25):
    """(sum of squared errors, sum of squared oracle values) over the full
    matrix of a homocorrelation given as packed upper-triangle planes (each
    entry off the diagonal stands for two), in FP64 on the planes' device."""
    num = den = 0.0
    for a in range(0, o.numel(), chunk):
        b = min(o.numel(), a + chunk)
        d = g[a:b].double() - o[a:b]
        num += float((d * d).sum())
        den += float((o[a:b] * o[a:b]).sum())
    dd = g[diag].double() - o[diag]
    num = 2.0 * num - float((dd * dd).sum())
    den = 2.0 * den - float((o[diag] * o[diag]).sum())
    return num, den


def full_rel_err(torch, g, o, diag):
    num, den = full_counts(torch, g, o, diag)
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


# Table 1 of the paper (Sec. 4.3): mean time of one corr2d() homocorrelation
# in seconds, R package corr2D 0.1.12 on an Intel Core i5-2450M (Windows 7),
# by cores and m, for n = 200, 400, 600, 1000, 4000, 8000.  Context only:
# other hardware, FP64 complex arithmetic, full n x n result.
TABLE1_N = (200, 400, 600, 1000, 4000, 8000)
TABLE1_S = {
    1: {5: (0.36, 0.50, 0.65, 1.05, 5.55, 16.37), 10: (0.36, 0.50, 0.66, 1.10, 5.76, 18.21),
        20: (0.36, 0.50, 0.67, 1.11, 6.17, 18.61), 100: (0.63, 0.98, 0.92, 1.33, 9.74, 33.04),
        500: (0.48, 0.82, 1.23, 2.57, 26.53, 105.23)},
    2: {5: (0.56, 0.69, 0.80, 1.18, 5.03, 15.09), 10: (0.62, 0.69, 0.83, 1.18, 5.16, 15.88),
        20: (0.56, 0.68, 0.82, 1.21, 5.40, 16.87), 100: (0.59, 0.73, 0.89, 1.33, 7.50, 27.01),
        500: (0.66, 0.92, 1.27, 2.15, 18.46, 74.43)},
    4: {5: (1.00, 1.11, 1.21, 1.62, 5.45, 15.49), 10: (0.99, 1.09, 1.22, 1.59, 5.55, 16.11),
        20: (0.99, 1.09, 1.23, 1.63, 5.88, 17.20), 100: (1.02, 1.13, 1.31, 1.73, 7.82, 26.81),
        500: (1.10, 1.42, 1.70, 2.62, 18.33, 72.34)},
}


def paper_context():
    """The paper's fastest whole-call rate (n^2 entries of the full complex
    matrix per second), for context next to this GPU's numbers."""
    best = None
    for cores, rows in TABLE1_S.items():
        for m, secs in rows.items():
            for n, sec in zip(TABLE1_N, secs):
                r = n * n / sec
                if best is None or r > best[0]:
                    best = (r, cores, m, n, sec)
    r, cores, m, n, sec = best
    return {"entries_per_s": r, "definition": "n^2 / mean corr2d() time (full complex matrix)",
            "config": f"m={m}, n={n}, {cores} cores, {sec} s",
            "hardware": "Intel Core i5-2450M, R corr2D 0.1.12, FP64 (Table 1 of the paper)",
            "kind": "context, not the target"}


def table1_sweep(B, torch, synth, dev, reps=5):
    """The paper's Table 1 grid on this GPU: full n x n homocorrelation, FP64
    and FP32 (whole call, inputs resident), next to the paper's seconds.
    Inputs: seeded band spectra (8 Lorentzians), a stand-in for the paper's
    simulated reaction data, whose parameters it does not give."""
    out = []
    for m in (5, 10, 20, 100, 500):
        for ni, n in enumerate(TABLE1_N):
            S, _ = synth.bands(m, n, 8, seed=synth.BASE_SEED + 20000 + 10 * m + ni)
            y = torch.as_tensor(S, device=dev)
            for prec in ("f64", "f32"):
                out_dtype = "f64" if prec == "f64" else "f32"
                plan = B.Plan(m=m, n1=n, n2=0, prec=prec, out_layout="full", in_dtype="f64",
                              out_dtype=out_dtype)
                tdt = torch.float64 if prec == "f64" else torch.float32
                phi = torch.empty(n * n, dtype=tdt, device=dev)
                psi = torch.empty(n * n, dtype=tdt, device=dev)
                ws = plan.workspace(dev)
                B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
                torch.cuda.synchronize()
                sec = (time.perf_counter() - t0) / reps
                paper = {c: TABLE1_S[c][m][ni] for c in TABLE1_S}
                out.append({"m": m, "n": n, "prec": prec, "ms_per_call": sec * 1e3,
                            "paper_s": paper, "ratio_to_best_paper": min(paper.values()) / sec})
                del phi, psi, ws, plan
            torch.cuda.empty_cache()
    return out


LAYOUT_TEXT = {"upper_aligned": "rows aligned to 128 bytes",
               "upper_packed": "packed rows"}


def run_variant(B, torch, y, n, m, prec, basis, steps, warmup, ev, ref,
                layout="upper_packed", alpha=0.0, flags=0):
    """Time `steps` calls; returns a dict of measurements for this form, with
    its error against the oracle over the full matrices.  ref = (oracle Phi,
    oracle Psi, diagonal positions, aligned-layout gather index), the oracle's
    values packed as upper triangles on the GPU."""
    out_dtype = "f64" if prec == "f64" else "f32"
    plan = B.Plan(m=m, n1=n, n2=0, prec=prec, basis=basis, out_layout=layout,
                  in_dtype="f64", out_dtype=out_dtype, scale_alpha=alpha, flags=flags)
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    numel = B.out_elements(layout, n)
    phi = torch.empty(numel, dtype=tdt, device=y.device)
    psi = torch.empty(numel, dtype=tdt, device=y.device)
    ws = plan.workspace(y.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        B.corr2d_homo(plan.handle, y, None, phi, psi, ws, stream=stream)
    evs = ev.create(2 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        B.corr2d_set_timing_events(evs[2 * s], evs[2 * s + 1])
        B.corr2d_homo(plan.handle, y, None, phi, psi, ws, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.corr2d_set_timing_events(None, None)
    kms = [ev.elapsed_ms(evs[2 * s], evs[2 * s + 1]) for s in range(steps)]
    ev.destroy(evs)
    o_phi, o_psi, diag, a2p = ref
    if layout == "upper_packed":
        err_phi = full_rel_err(torch, phi, o_phi, diag)
        err_psi = full_rel_err(torch, psi, o_psi, diag)
    else:
        err_phi = full_rel_err(torch, phi[a2p], o_phi, diag)
        err_psi = full_rel_err(torch, psi[a2p], o_psi, diag)
    info = plan.info
    entries = n * (n + 1) // 2
    alg_flops = 4.0 * m * entries
    executed = 2.0 * 2.0 * info.tiles * info.tile_m * info.tile_n * info.k_pad
    sel = B.selection(ws, plan)
    if sel is not None:
        # hi*hi over every K block, hi*lo and lo*hi over the selected ones
        executed *= 1 + 2 * sel[0] / len(sel[1])
    elif prec in ("split_bf16", "split_f16"):
        executed *= 3
    kernel_ms = float(np.mean(kms))
    esz = 8 if out_dtype == "f64" else 4
    planes = {"f64": 8, "f32": 4, "split_bf16": 4, "bf16": 2, "f16": 2, "fp8_e4m3": 1,
              "split_f16": 4}[prec]
    kernel_bytes = 2 * entries * esz + 2 * n * info.k_pad * planes
    res = {
        "prec": prec, "basis": {v: k for k, v in B.BASIS.items()}[plan.info.basis],
        "scale_alpha": alpha, "layout": layout,
        "ms_per_step": wall * 1e3 / steps,
        "entries_per_s": entries / (wall / steps),
        "kernel_ms": kernel_ms,
        "kernel_alg_tflops": alg_flops / (kernel_ms * 1e-3) / 1e12,
        "kernel_executed_tflops": executed / (kernel_ms * 1e-3) / 1e12,
        # executed MFMA rate against the dense peak of the precision issued
        "mfma_peak_tflops": PEAK_TFLOPS[prec],
        "mfma_executed_frac": executed / (kernel_ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
        "kernel_hbm_GBps": kernel_bytes / (kernel_ms * 1e-3) / 1e9,
        "err_phi": err_phi,
        "err_psi": err_psi,
        "tile": f"{info.tile_m}x{info.tile_n}",
        "row_select": None if sel is None else {"split_k_blocks": sel[0], "k_blocks": len(sel[1])},
        "alg_flops": alg_flops, "executed_flops": executed, "kernel_bytes": kernel_bytes,
    }
    del phi, psi, ws, plan
    torch.cuda.empty_cache()
    return res


def kernel_code_sha256(path):
    """SHA-256 of a source file with its comments removed and whitespace
    collapsed: the counters stay valid across edits that change no code."""
    import hashlib
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    src = " ".join(src.split())   # layout-only edits do not count either
    return hashlib.sha256(src.encode()).hexdigest()


def profile_record(kernel_tag="corr2_split_m256_n16384"):
    """The committed PMC record of the contraction kernel (HBM bytes from
    FETCH_SIZE and WRITE_SIZE, each scaled by a 1 GiB copy; MFMA operations
    from SQ_INSTS_VALU_MFMA_MOPS_BF16), or None when the kernel code has
    changed since the counters were taken."""
    rec_path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    src = os.path.join(ROOT, "paper_1808_00685_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(rec_path))
        sha = kernel_code_sha256(src)
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_code_sha256") != sha:
        return None
    return rec


def cpu_baseline(oracle, S, target_s):
    """The oracle's direct route on a bounded sample of output rows: calls on
    doubling row counts until one takes about a third of the target, then
    one call sized to the target from that call's rate (reported)."""
    Y, _ = oracle.dynamic(S)
    m, n = Y.shape
    rows = 256
    while True:
        t0 = time.perf_counter()
        oracle.corr_ht(Y[:, :rows], Y)
        dt = time.perf_counter() - t0
        if dt >= target_s / 3 or rows >= n:
            break
        rows = min(n, rows * 2)
    calls = 1
    if rows < n:
        rows = int(min(n, max(rows, rows * target_s / dt)))
    else:
        # the whole matrix is quicker than the target: repeat it
        calls = max(1, int(round(target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(calls):
        oracle.corr_ht(Y[:, :rows], Y)
    dt = time.perf_counter() - t0
    return {"value": calls * rows * n / dt, "unit": "entries/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"direct route (FP64, OpenMP) for the first {rows} spectral points "
                      f"against all {n} of the m={m} x n={n} workload, {calls} call(s): "
                      f"{calls * rows * n} (Phi, Psi) entries in {dt:.1f} s"}


def host_cpu():
    """The host's CPU model, logical CPUs and the CPUs this process may use."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def time_calls(torch, fn, reps, batches=3):
    """Wall time per call of `reps` back-to-back calls (ms), the fastest of
    `batches` batches: one host-side hiccup of a few ms would otherwise
    double the figure of a sub-millisecond call."""
    fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(batches):
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3 / reps
        best = t if best is None else min(best, t)
    return best


def kernel_ms(B, torch, plan, call, ev, reps=7):
    """Median contraction-kernel time (ms) of `reps` calls through the
    library's timing hook.  The median, not the mean: when the host is late
    to submit the kernel after the event before it, that one interval
    includes the wait, and a mean over a few calls of a 40 us kernel takes
    it in whole."""
    evs = ev.create(2 * reps)
    for r in range(reps):
        B.corr2d_set_timing_events(evs[2 * r], evs[2 * r + 1])
        call()
    torch.cuda.synchronize()
    ms = [ev.elapsed_ms(evs[2 * r], evs[2 * r + 1]) for r in range(reps)]
    B.corr2d_set_timing_events(None, None)
    ev.destroy(evs)
    return float(np.median(ms))


def timed_oracle(oracle, fn, threads=None):
    """Run fn() on the oracle (with `threads` OpenMP threads if given) and
    return (result, seconds)."""
    all_threads = oracle.threads()
    if threads is not None:
        oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        r = fn()
        return r, time.perf_counter() - t0
    finally:
        oracle.set_threads(all_threads)


def other_workloads(B, torch, oracle, synth, ev, dev):
    """The other workload configurations: small FP64 (latency), medium full
    FP32/FP64 (output-bound), heterocorrelation FP16/FP8 (output-bound) and
    the batch of 256 data sets (persistent graph against sequential
    launches), each with its error against the oracle over the full
    matrices.  Also returns the oracle's own times on these workloads."""
    out, otimes = [], []
    nthreads = oracle.threads()

    # small: m = 11, n = 512, FP64, full output
    S, _ = synth.workload_small()
    m, n = S.shape
    y = torch.as_tensor(S, device=dev)
    plan = B.Plan(m=m, n1=n, n2=0, prec="f64", in_dtype="f64", out_dtype="f64")
    phi = torch.empty(n * n, dtype=torch.float64, device=dev)
    psi = torch.empty(n * n, dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)
    call = lambda: B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
    ms = time_calls(torch, call, 50)
    (po, qo), t_all = timed_oracle(oracle, lambda: oracle.corr2d(S))
    _, t_one = timed_oracle(oracle, lambda: oracle.corr2d(S), threads=1)
    for th, t in ((nthreads, t_all), (1, t_one)):
        otimes.append({"workload": f"m={m} n={n}, full", "threads": th, "seconds": t,
                       "entries_per_s": n * n / t})
    out.append({"workload": f"homocorrelation m={m} n={n}, FP64, full output", "prec": "f64",
                "ms_per_call": ms, "entries_per_s": n * n / (ms * 1e-3),
                "err_phi": rel_fro(phi.cpu().numpy().reshape(n, n), po),
                "err_psi": rel_fro(psi.cpu().numpy().reshape(n, n), qo),
                "error_measure": "relative Frobenius, full matrices"})
    del plan, phi, psi, ws

    # medium: m = 64, n = 4096, FP32 and FP64, full output (mirror stored)
    S, meta = synth.workload_medium()
    m, n = S.shape
    y = torch.as_tensor(S, device=dev)
    (po, qo), t_all = timed_oracle(oracle, lambda: oracle.corr2d(S))
    _, t_one = timed_oracle(oracle, lambda: oracle.corr2d(S), threads=1)
    for th, t in ((nthreads, t_all), (1, t_one)):
        otimes.append({"workload": f"m={m} n={n}, full", "threads": th, "seconds": t,
                       "entries_per_s": n * n / t})
    po_t, qo_t = torch.as_tensor(po, device=dev), torch.as_tensor(qo, device=dev)
    del po, qo
    for prec in ("f32", "f64"):
        tdt = torch.float64 if prec == "f64" else torch.float32
        plan = B.Plan(m=m, n1=n, n2=0, prec=prec, in_dtype="f64", out_dtype=prec)
        phi = torch.empty(n * n, dtype=tdt, device=dev)
        psi = torch.empty(n * n, dtype=tdt, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
        ms = time_calls(torch, call, 20)
        kms = kernel_ms(B, torch, plan, call, ev)
        nbytes = 2 * n * n * (8 if prec == "f64" else 4)
        out.append({"workload": f"homocorrelation m={m} n={n}, full output", "prec": prec,
                    "ms_per_call": ms, "entries_per_s": n * n / (ms * 1e-3), "kernel_ms": kms,
                    "roofline": {"bound": "hbm", "achieved": nbytes / (kms * 1e-3) / 1e9,
                                 "peak": HBM_GBPS, "unit": "GB/s",
                                 "frac": nbytes / (kms * 1e-3) / 1e9 / HBM_GBPS,
                                 "bytes_per_launch": nbytes},
                    "err_phi": float(torch.linalg.norm(phi.double() - po_t.ravel()) / torch.linalg.norm(po_t)),
                    "err_psi": float(torch.linalg.norm(psi.double() - qo_t.ravel()) / torch.linalg.norm(qo_t)),
                    "error_measure": "relative Frobenius, full matrices"})
        del plan, phi, psi, ws
    del po_t, qo_t

    # heterocorrelation: m = 128, n1 = 8192, n2 = 2048, FP16 and FP8, full output
    S1, S2, meta = synth.workload_hetero()
    m, n1 = S1.shape
    n2 = S2.shape[1]
    y1 = torch.as_tensor(S1, device=dev)
    y2 = torch.as_tensor(S2, device=dev)
    (po, qo), t_all = timed_oracle(oracle, lambda: oracle.corr2d(S1, S2=S2))
    otimes.append({"workload": f"hetero m={m} n1={n1} n2={n2}, full", "threads": nthreads,
                   "seconds": t_all, "entries_per_s": n1 * n2 / t_all})
    po_t, qo_t = torch.as_tensor(po, device=dev).ravel(), torch.as_tensor(qo, device=dev).ravel()
    del po, qo
    for prec in ("f16", "fp8_e4m3", "split_bf16"):
        plan = B.Plan(m=m, n1=n1, n2=n2, prec=prec, in_dtype="f64", out_dtype="f32")
        phi = torch.empty(n1 * n2, dtype=torch.float32, device=dev)
        psi = torch.empty(n1 * n2, dtype=torch.float32, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_hetero(plan.handle, y1, None, y2, None, phi, psi, ws)
        ms = time_calls(torch, call, 20)
        kms = kernel_ms(B, torch, plan, call, ev)
        nbytes = 2 * n1 * n2 * 4
        out.append({"workload": f"heterocorrelation m={m} n1={n1} n2={n2}, full output",
                    "prec": prec, "ms_per_call": ms, "entries_per_s": n1 * n2 / (ms * 1e-3),
                    "kernel_ms": kms,
                    "roofline": {"bound": "hbm", "achieved": nbytes / (kms * 1e-3) / 1e9,
                                 "peak": HBM_GBPS, "unit": "GB/s",
                                 "frac": nbytes / (kms * 1e-3) / 1e9 / HBM_GBPS,
                                 "bytes_per_launch": nbytes},
                    "err_phi": float(torch.linalg.norm(phi.double() - po_t) / torch.linalg.norm(po_t)),
                    "err_psi": float(torch.linalg.norm(psi.double() - qo_t) / torch.linalg.norm(qo_t)),
                    "error_measure": "relative Frobenius, full matrices"})
        del plan, phi, psi, ws
    del po_t, qo_t

    # batch of 256 data sets, FP32 and split-BF16, upper triangles
    out.extend(batch_workload(B, torch, oracle, synth, dev, otimes))
    torch.cuda.empty_cache()
    return out, otimes


def batch_workload(B, torch, oracle, synth, dev, otimes):
    """The batch of 256 data sets: one graph replay of the persistent launch
    (FP32 and split-BF16) and the FP32 sequential launches, timed; then every
    data set's full Phi and Psi against the oracle (per-set relative
    Frobenius errors; the worst set and the whole batch are reported)."""
    items = synth.batch_spec()
    data = [synth.batch_item_data(it) for it in items]
    offs, ooffs, cur, ocur = [], [], 0, 0
    for it in items:
        offs.append(cur)
        ooffs.append(ocur)
        cur += it.m * it.n
        ocur += it.n * (it.n + 1) // 2
    y = torch.empty(cur, dtype=torch.float64, device=dev)
    for it, Sd, o in zip(items, data, offs):
        y[o:o + it.m * it.n] = torch.as_tensor(Sd.ravel(), device=dev)
    spec = [(it.m, it.n, o, 0, oo) for it, o, oo in zip(items, offs, ooffs)]
    res, outs = {}, {}
    for name, prec, flags in (("graph", "f32", 0), ("sequential", "f32", B.FLAG_SEQUENTIAL),
                              ("split", "split_bf16", 0), ("split16", "split_f16", 0)):
        if name != "sequential":
            outs[name] = (torch.empty(ocur, dtype=torch.float32, device=dev),
                          torch.empty(ocur, dtype=torch.float32, device=dev))
        phi, psi = outs["graph" if name == "sequential" else name]
        plan = B.Plan(B.corr2d_desc_init(prec=prec, out_layout="upper_packed", flags=flags),
                      items=spec)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_batched(plan.handle, y, phi, psi, ws)
        res[name] = time_calls(torch, call, 5)
        del plan, ws
    del y
    # every set's upper triangle against the oracle's
    agg = {k: [0.0, 0.0, 0.0, 0.0] for k in outs}
    worst = {k: (0.0, -1, 0.0, 0.0) for k in outs}
    osecs = 0.0
    for k, (it, Sd, oo) in enumerate(zip(items, data, ooffs)):
        o_phi, o_psi, secs = upper_oracle(oracle, torch, Sd, dev)
        osecs += secs
        diag = packed_diag(torch, it.n, dev)
        tot = it.n * (it.n + 1) // 2
        for name, (phi, psi) in outs.items():
            c_phi = full_counts(torch, phi[oo:oo + tot], o_phi, diag)
            c_psi = full_counts(torch, psi[oo:oo + tot], o_psi, diag)
            a = agg[name]
            a[0] += c_phi[0]; a[1] += c_phi[1]; a[2] += c_psi[0]; a[3] += c_psi[1]
            e_phi = math.sqrt(c_phi[0] / c_phi[1]) if c_phi[1] > 0 else math.sqrt(c_phi[0])
            e_psi = math.sqrt(c_psi[0] / c_psi[1]) if c_psi[1] > 0 else math.sqrt(c_psi[0])
            if max(e_phi, e_psi) > max(worst[name][2], worst[name][3]):
                worst[name] = (0.0, k, e_phi, e_psi)
        del o_phi, o_psi
    entries = sum(it.n * (it.n + 1) // 2 for it in items)
    alg_flops = sum(4.0 * it.m * it.n * (it.n + 1) / 2 for it in items)
    out_bytes = 8.0 * entries                                    # both FP32 planes
    in_bytes = sum(8.0 * it.m * it.n for it in items)            # FP64 spectra read once
    otimes.append({"workload": f"batch of {len(items)} sets, upper triangles", "threads": oracle.threads(),
                   "seconds": osecs, "entries_per_s": entries / osecs})
    desc = f"batch of {len(items)} homocorrelations, m in 8..200, n in 256..8192, "
    rows = []
    for name, prec, text in (("graph", "f32", "FP32"), ("split", "split_bf16", "split-BF16"),
                             ("split16", "split_f16", "split-FP16")):
        a, w = agg[name], worst[name]
        r = {"workload": desc + text + ", upper triangles", "prec": prec,
             "ms_per_call": res[name], "entries_per_s": entries / (res[name] * 1e-3),
             "err_phi": math.sqrt(a[0] / a[1]), "err_psi": math.sqrt(a[2] / a[3]),
             "worst_set": {"index": w[1], "m": items[w[1]].m, "n": items[w[1]].n,
                           "err_phi": w[2], "err_psi": w[3]},
             "error_measure": "relative Frobenius over all data sets' full matrices; "
                              "worst_set: the largest per-set error"}
        # the whole batch's roofline (one call): the algorithm's intensity
        # (4m flops per 8 stored bytes) is above the FP32 ridge (157.3/8 flop/B)
        # and below the 16-bit one (2500/8): FP32 is bound by its MFMA peak,
        # the split forms by HBM
        sec = res[name] * 1e-3
        if prec == "f32":
            ach = alg_flops / sec / 1e12
            r["roofline"] = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["f32"],
                             "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["f32"],
                             "algorithmic_flops_per_call": alg_flops}
        else:
            ach = (out_bytes + in_bytes) / sec / 1e9
            r["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_GBPS, "unit": "GB/s",
                             "frac": ach / HBM_GBPS, "algorithmic_bytes_per_call": out_bytes + in_bytes}
        if name == "graph":
            r["sequential_ms_per_call"] = res["sequential"]
            r["graph_speedup"] = res["sequential"] / res["graph"]
        rows.append(r)
    del outs
    return rows


def profile_run(B, torch, synth, dev, spec, reps):
    """Only the calls of one workload, for profiler runs (--profile
    WORKLOAD:PREC[:rowsel]); prints one JSON line with the mean wall time."""
    parts = spec.split(":")
    work, prec = parts[0], parts[1]
    flags = B.FLAG_SPLIT_ROWS if "rowsel" in parts[2:] else 0
    out_dtype = "f64" if prec == "f64" else "f32"
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    if work == "large":
        S, _ = synth.workload_large()
        m, n = S.shape
        y = torch.as_tensor(S, device=dev)
        plan = B.Plan(m=m, n1=n, n2=0, prec=prec, out_layout="upper_aligned", in_dtype="f64",
                      out_dtype=out_dtype, flags=flags)
        numel = B.out_elements("upper_aligned", n)
        phi = torch.empty(numel, dtype=tdt, device=dev)
        psi = torch.empty(numel, dtype=tdt, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
    elif work == "medium":
        S, _ = synth.workload_medium()
        m, n = S.shape
        y = torch.as_tensor(S, device=dev)
        plan = B.Plan(m=m, n1=n, n2=0, prec=prec, in_dtype="f64", out_dtype=out_dtype, flags=flags)
        phi = torch.empty(n * n, dtype=tdt, device=dev)
        psi = torch.empty(n * n, dtype=tdt, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
    elif work == "hetero":
        S1, S2, _ = synth.workload_hetero()
        y1, y2 = torch.as_tensor(S1, device=dev), torch.as_tensor(S2, device=dev)
        n1, n2 = S1.shape[1], S2.shape[1]
        plan = B.Plan(m=S1.shape[0], n1=n1, n2=n2, prec=prec, in_dtype="f64", out_dtype=out_dtype,
                      flags=flags)
        phi = torch.empty(n1 * n2, dtype=tdt, device=dev)
        psi = torch.empty(n1 * n2, dtype=tdt, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_hetero(plan.handle, y1, None, y2, None, phi, psi, ws)
    elif work == "batch":
        items = synth.batch_spec()
        offs, ooffs, cur, ocur = [], [], 0, 0
        for it in items:
            offs.append(cur)
            ooffs.append(ocur)
            cur += it.m * it.n
            ocur += it.n * (it.n + 1) // 2
        y = torch.empty(cur, dtype=torch.float64, device=dev)
        for it, o in zip(items, offs):
            y[o:o + it.m * it.n] = torch.as_tensor(synth.batch_item_data(it).ravel(), device=dev)
        plan = B.Plan(B.corr2d_desc_init(prec=prec, out_layout="upper_packed", flags=flags),
                      items=[(it.m, it.n, o, 0, oo) for it, o, oo in zip(items, offs, ooffs)])
        phi = torch.empty(ocur, dtype=torch.float32, device=dev)
        psi = torch.empty(ocur, dtype=torch.float32, device=dev)
        ws = plan.workspace(dev)
        call = lambda: B.corr2d_batched(plan.handle, y, phi, psi, ws)
    else:
        raise SystemExit(f"unknown workload {work}")
    ms = time_calls(torch, call, reps, batches=1)
    print(json.dumps({"profile": spec, "ms_per_call": ms, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--layout", default="upper_aligned", choices=["upper_aligned", "upper_packed"],
                    help="storage of the upper triangle in the headline line")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the benchmark line, time the paper's Table 1 grid (FP64, FP32)")
    ap.add_argument("--profile", metavar="WORKLOAD:PREC[:rowsel]",
                    help="instead of the benchmark line, only call one workload (large, medium, "
                         "hetero, batch) --steps times, for profiler runs")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the contraction shards by output tiles with no collective, see DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1808_00685_amd import binding as B
    from paper_1808_00685_amd import synth
    from paper_1808_00685_amd.timing import HipEvents

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    if args.profile:
        profile_run(B, torch, synth, dev, args.profile, args.steps)
        return
    if args.table1:
        print(json.dumps({"table1": table1_sweep(B, torch, synth, dev), "paper": paper_context()}),
              flush=True)
        return
    m, n = args.m, args.n
    S, meta = synth.workload_large(m=m, n=n)
    y = torch.as_tensor(S, device=dev)
    ev = HipEvents()
    # the oracle over the whole upper triangle (outside every timed region)
    o_phi, o_psi, c3_secs = upper_oracle(oracle, torch, S, dev)
    diag = packed_diag(torch, n, dev)
    a2p = aligned_to_packed_index(torch, n, dev)
    ref = (o_phi, o_psi, diag, a2p)

    layout = args.layout
    main_res = run_variant(B, torch, y, n, m, "split_bf16", "auto", args.steps, args.warmup,
                           ev, ref, layout=layout)
    variants = []
    if not args.no_variants:
        vs = args.variant_steps
        # the headline form in the other upper-triangle layout
        other = "upper_packed" if layout == "upper_aligned" else "upper_aligned"
        variants.append(run_variant(B, torch, y, n, m, "split_bf16", "auto", vs, 1, ev, ref,
                                    layout=other))
        # the headline form in the Fourier basis (the default is the time
        # basis), and the other formats
        for prec, basis in (("split_bf16", "fourier"), ("split_f16", "auto"), ("f32", "auto"),
                            ("bf16", "fourier"), ("bf16", "auto"), ("f64", "auto")):
            variants.append(run_variant(B, torch, y, n, m, prec, basis, vs, 1, ev, ref,
                                        layout=layout))
        # the row-selective split (low plane on the high-energy Fourier rows
        # only; target 1e-5)
        for prec in ("split_bf16", "split_f16"):
            variants.append(run_variant(B, torch, y, n, m, prec, "fourier", vs, 1, ev, ref,
                                        layout=layout, flags=B.FLAG_SPLIT_ROWS))
        # Pareto scaling (alpha = 0.5) of the headline form: the oracle's
        # values times its scaling factors (oracle.corr2d's alpha)
        f = torch.as_tensor(oracle.scaling_factors(oracle.band_sd(oracle.dynamic(S)[0]), 0.5),
                            device=dev)
        ii = torch.arange(n, device=dev, dtype=torch.int64)
        rows = torch.repeat_interleave(ii, n - ii)
        cols = torch.arange(rows.numel(), device=dev, dtype=torch.int64) - diag[rows] + rows
        w = f[rows] * f[cols]
        del rows, cols
        pref = (o_phi * w, o_psi * w, diag, a2p)
        del w
        variants.append(run_variant(B, torch, y, n, m, "split_bf16", "auto", vs, 1, ev, pref,
                                    alpha=0.5, layout=layout))
        del pref
    del ref, o_phi, o_psi, a2p
    torch.cuda.empty_cache()

    workloads, otimes = [], []
    if not args.no_workloads:
        workloads, otimes = other_workloads(B, torch, oracle, synth, ev, dev)
    otimes.insert(0, {"workload": f"m={m} n={n}, upper triangle", "threads": oracle.threads(),
                      "seconds": c3_secs, "entries_per_s": n * (n + 1) // 2 / c3_secs})

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(oracle, S, args.cpu_seconds)
        cpu["host"] = host_cpu()
        cpu["per_workload"] = otimes

    prof = profile_record() if (m, n, layout) == (256, 16384, "upper_aligned") else None
    alg = main_res["alg_flops"]
    kms = main_res["kernel_ms"]
    achieved = alg / (kms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": main_res["entries_per_s"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "split-bf16",
        "data": "synthetic",
        "config": {"workload": f"homocorrelation m={m} n={n} band spectra, upper triangle "
                               f"({LAYOUT_TEXT[layout]}), FP32 output, time basis, Noda kernel",
                   "m": m, "n": n, "layout": layout, "prec": "split_bf16",
                   "entries_per_step": n * (n + 1) // 2},
        # The algorithm's intensity (4m flops per 8 written bytes, plus the
        # operands read once) is below the BF16 ridge (2500/8 flop/B), so the
        # roof is HBM; the MFMA figures (algorithmic, and executed with the
        # split form's three products) ride along.
        "roofline": {
            "bound": "hbm", "kernel": f"corr2_kernel<split_bf16> ({main_res['tile']} tiles)",
            "achieved": main_res["kernel_hbm_GBps"], "peak": HBM_GBPS, "unit": "GB/s",
            "frac": main_res["kernel_hbm_GBps"] / HBM_GBPS,
            "traffic": (prof or {}).get("traffic_bytes_per_launch"),
            "executed_flops_counted": (prof or {}).get("executed_mfma_flops_counted"),
            "kernel_ms": kms,
            "algorithmic_bytes_per_launch": main_res["kernel_bytes"],
            "algorithmic_flops_per_launch": alg,
            "intensity_flop_per_byte": alg / main_res["kernel_bytes"],
            "bf16_ridge_flop_per_byte": PEAK_TFLOPS["split_bf16"] / HBM_GBPS * 1e3,
            "mfma_alg_tflops": achieved,
            "mfma_alg_frac": achieved / PEAK_TFLOPS["split_bf16"],
            "executed_tflops": main_res["kernel_executed_tflops"],
            "executed_frac": main_res["kernel_executed_tflops"] / PEAK_TFLOPS["split_bf16"],
        },
        "error_vs_oracle": {"phi": main_res["err_phi"], "psi": main_res["err_psi"],
                            "measure": "relative Frobenius over the full n x n matrices "
                                       f"({n * (n + 1) // 2} stored entries compared)"},
        "cpu_baseline": cpu,
        "paper_context": paper_context(),
        "variants": [{k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in r.items()
                      if k not in ("alg_flops", "executed_flops", "kernel_bytes")}
                     for r in variants],
        "workloads": workloads,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
