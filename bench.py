#!/usr/bin/env python3
"""Benchmark of the generalized 2D correlation hot path on one MI355X.

One step = one corr2d_homo call through the C ABI on the m=256 x n=16384
band workload (128 Lorentzian/Gaussian bands, amplitudes 1e-3..1e2, noise
1e-4; upper triangle stored, FP32 output): FP64 centring, transform tables,
FP32 MFMA transform to split-BF16 Fourier operands, split-BF16 MFMA
contraction with FP64 epilogue.  Inputs are resident in HBM before timing.

Prints ONE JSON line: throughput in correlation entries/s (stored
(Phi, Psi) pairs), the roofline of the contraction kernel (timed alone with
HIP events on the call's stream through the library's timing hook), the
error against the FP64 oracle on sampled entries, the same measurements for
the plain FP32, FP64 and BF16 forms, and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import ctypes
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
               "f16": 2500.0, "fp8_e4m3": 5000.0}
HBM_GBPS = 8000.0


class HipEvents:
    """hipEvent_t handles through libamdhip64 (the library records them on
    the stream its kernels run on)."""

    def __init__(self):
        self.h = ctypes.CDLL("libamdhip64.so")
        self.h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.h.hipEventSynchronize.argtypes = [ctypes.c_void_p]

    def create(self, n):
        evs = []
        for _ in range(n):
            e = ctypes.c_void_p()
            assert self.h.hipEventCreate(ctypes.byref(e)) == 0
            evs.append(e.value)
        return evs

    def elapsed_ms(self, a, b):
        self.h.hipEventSynchronize(b)
        t = ctypes.c_float()
        assert self.h.hipEventElapsedTime(ctypes.byref(t), a, b) == 0
        return float(t.value)

    def destroy(self, evs):
        for e in evs:
            self.h.hipEventDestroy(e)


def sample_pairs(n, count, seed, centers):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    c = np.unique(np.clip(np.round(centers).astype(np.int64), 0, n - 1))
    ci, cj = np.meshgrid(c, c, indexing="ij")
    i = np.concatenate([i, ci.ravel()])
    j = np.concatenate([j, cj.ravel()])
    return np.minimum(i, j).astype(np.int64), np.maximum(i, j).astype(np.int64)


def rel_fro(g, o):
    return float(np.linalg.norm(g - o) / np.linalg.norm(o))


def run_variant(B, torch, y, n, m, prec, basis, steps, warmup, ev, sample, oracle_vals,
                layout="upper_packed"):
    """Time `steps` calls; returns a dict of measurements for this form."""
    out_dtype = "f64" if prec == "f64" else "f32"
    plan = B.Plan(m=m, n1=n, n2=0, prec=prec, basis=basis, out_layout=layout,
                  in_dtype="f64", out_dtype=out_dtype)
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    numel = n * (n + 1) // 2
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
        B.corr2d_plan_set_timing_events(plan.handle, evs[2 * s], evs[2 * s + 1])
        B.corr2d_homo(plan.handle, y, None, phi, psi, ws, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.corr2d_plan_set_timing_events(plan.handle, None, None)
    kms = [ev.elapsed_ms(evs[2 * s], evs[2 * s + 1]) for s in range(steps)]
    ev.destroy(evs)
    i, j = sample
    idx = torch.as_tensor(i * n - (i * (i - 1)) // 2 + (j - i), device=y.device)
    g_phi = phi[idx].double().cpu().numpy()
    g_psi = psi[idx].double().cpu().numpy()
    info = plan.info
    entries = n * (n + 1) // 2
    alg_flops = 4.0 * m * entries
    executed = 2.0 * 2.0 * info.tiles * info.tile_m * info.tile_n * info.k_pad
    if prec == "split_bf16":
        executed *= 3
    kernel_ms = float(np.mean(kms))
    esz = 8 if out_dtype == "f64" else 4
    planes = {"f64": 8, "f32": 4, "split_bf16": 4, "bf16": 2, "f16": 2, "fp8_e4m3": 1}[prec]
    kernel_bytes = 2 * entries * esz + 2 * n * info.k_pad * planes
    res = {
        "prec": prec, "basis": basis,
        "ms_per_step": wall * 1e3 / steps,
        "entries_per_s": entries / (wall / steps),
        "kernel_ms": kernel_ms,
        "kernel_alg_tflops": alg_flops / (kernel_ms * 1e-3) / 1e12,
        "kernel_executed_tflops": executed / (kernel_ms * 1e-3) / 1e12,
        "kernel_hbm_GBps": kernel_bytes / (kernel_ms * 1e-3) / 1e9,
        "err_phi": rel_fro(g_phi, oracle_vals[0]),
        "err_psi": rel_fro(g_psi, oracle_vals[1]),
        "tile": f"{info.tile_m}x{info.tile_n}",
        "alg_flops": alg_flops, "executed_flops": executed, "kernel_bytes": kernel_bytes,
    }
    del phi, psi, ws, plan
    torch.cuda.empty_cache()
    return res


def measured_traffic(kernel_tag="corr2_split_m256_n16384"):
    """HBM bytes per launch of the contraction kernel from the committed PMC
    record (FETCH_SIZE and WRITE_SIZE, each scaled by a 1 GiB copy), or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    src = os.path.join(ROOT, "paper_1808_00685_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(rec_path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != sha:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(oracle, S, target_s):
    """The oracle's direct route on a bounded sample of output rows."""
    Y, _ = oracle.dynamic(S)
    m, n = Y.shape
    # two short runs separate the per-row cost from the fixed cost (the
    # Hilbert-Noda transform of all columns), then one run of ~target_s
    times = {}
    for r in (32, 128):
        t0 = time.perf_counter()
        oracle.corr_ht(Y[:, :r], Y)
        times[r] = time.perf_counter() - t0
    per_row = max((times[128] - times[32]) / 96.0, 1e-6)
    fixed = max(times[32] - 32 * per_row, 0.0)
    rows = int(min(n, max(128, (target_s - fixed) / per_row)))
    t0 = time.perf_counter()
    oracle.corr_ht(Y[:, :rows], Y)
    dt = time.perf_counter() - t0
    return {"value": rows * n / dt, "unit": "entries/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"direct route (FP64, OpenMP) for the first {rows} spectral points "
                      f"against all {n} of the m={m} x n={n} workload: {rows * n} "
                      f"(Phi, Psi) entries in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--n", type=int, default=16384)
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

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    m, n = args.m, args.n
    S, meta = synth.workload_large(m=m, n=n)
    sample = sample_pairs(n, 3000, 5, meta["centers"][:48])
    oracle_vals = oracle.corr2d_entries(S, sample[0], sample[1])
    y = torch.as_tensor(S, device=dev)
    ev = HipEvents()

    main_res = run_variant(B, torch, y, n, m, "split_bf16", "fourier", args.steps, args.warmup,
                           ev, sample, oracle_vals)
    variants = []
    if not args.no_variants:
        vs = args.variant_steps
        for prec, basis in (("f32", "fourier"), ("bf16", "fourier"), ("bf16", "time"),
                            ("f64", "fourier")):
            variants.append(run_variant(B, torch, y, n, m, prec, basis, vs, 1, ev, sample,
                                        oracle_vals))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(oracle, S, args.cpu_seconds)

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
        "config": {"workload": f"homocorrelation m={m} n={n} band spectra, upper triangle, "
                               "FP32 output, Fourier basis, Noda kernel",
                   "m": m, "n": n, "layout": "upper_packed", "prec": "split_bf16",
                   "entries_per_step": n * (n + 1) // 2},
        "roofline": {
            "bound": "mfma", "kernel": f"corr2_kernel<split_bf16> ({main_res['tile']} tiles)",
            "achieved": achieved, "peak": PEAK_TFLOPS["split_bf16"], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS["split_bf16"],
            "traffic": measured_traffic() if (m, n) == (256, 16384) else None,
            "kernel_ms": kms,
            "algorithmic_flops_per_launch": alg,
            "executed_tflops": main_res["kernel_executed_tflops"],
            "executed_frac": main_res["kernel_executed_tflops"] / PEAK_TFLOPS["split_bf16"],
            "hbm_GBps": main_res["kernel_hbm_GBps"],
            "hbm_frac": main_res["kernel_hbm_GBps"] / HBM_GBPS,
        },
        "error_vs_oracle": {"phi": main_res["err_phi"], "psi": main_res["err_psi"],
                            "sampled_entries": int(len(sample[0]))},
        "cpu_baseline": cpu,
        "variants": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()
                      if k not in ("alg_flops", "executed_flops", "kernel_bytes")}
                     for r in variants],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
