"""Autotuner of the contraction tile shape (run on the GPU the table is for).

``python -m paper_1808_00685_amd.tune`` times the correlation kernel of every
tile shape built for each precision over a grid of size classes (perturbation
length m, spectral points n) and writes the winners as the rule table the
library reads at plan time (``tune/gfx950.tsv`` next to ``libcorr2d.so``, or
the file named by ``CORR2D_TUNE_TABLE``).  One rule per line::

    prec  m_max  n_max  tile

The library takes the first rule whose precision matches with m <= m_max and
n <= n_max, so the rules of a precision are written in increasing m_max, then
n_max, the last class of each axis open-ended.
"""
from __future__ import annotations

import argparse
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune", "gfx950.tsv")
OPEN = 1 << 40   # upper bound of the last size class

# tile ids built per precision (1: 64 x 64, 2: 128 x 128 or 256 x 128 for the
# 16-bit formats, 3: 128 x 128 of the LDS-staged kernel)
CANDIDATES = {
    "f64": [1, 2],
    "f32": [1, 2],
    "split_bf16": [2, 3],
    "bf16": [2, 3],
    "f16": [2, 3],
    "fp8_e4m3": [1, 2],
    "split_f16": [2, 3],
}
M_CLASSES = [16, 64, 256]
N_CLASSES = [512, 2048, 8192, 16384]


def rules_from_timings(timings):
    """timings: {(prec, m_class, n_class): {tile: ms}} -> table lines.

    Classes are bounded by the next larger class: the rule for (m_c, n_c)
    covers m <= m_c and n <= n_c; the largest class of each axis is
    open-ended."""
    from . import binding as B
    lines = []
    for prec in CANDIDATES:
        ms = sorted({k[1] for k in timings if k[0] == prec})
        ns = sorted({k[2] for k in timings if k[0] == prec})
        for mi, mc in enumerate(ms):
            for ni, nc in enumerate(ns):
                t = timings.get((prec, mc, nc))
                if not t:
                    continue
                best = min(t, key=t.get)
                m_max = OPEN if mi == len(ms) - 1 else mc
                n_max = OPEN if ni == len(ns) - 1 else nc
                lines.append(f"{B.PREC[prec]}\t{m_max}\t{n_max}\t{best}")
    return lines


def write_table(lines, path, header):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# prec\tm_max\tn_max\ttile\n")
        for h in header:
            f.write(f"# {h}\n")
        for ln in lines:
            f.write(ln + "\n")


def time_tile(B, torch, prec, m, n, tile, ev, reps=11):
    """Median contraction-kernel time (ms) of one homocorrelation plan (row-aligned
    upper triangle, the benchmark's layout)."""
    import numpy as np
    dev = torch.device("cuda:0")
    plan = B.Plan(m=m, n1=n, n2=0, prec=prec, out_layout="upper_aligned", in_dtype="f64",
                  out_dtype="f64" if prec == "f64" else "f32", tile=tile)
    y = torch.randn(m, n, dtype=torch.float64, device=dev) + 3.0
    numel = B.out_elements("upper_aligned", n)
    odt = torch.float64 if prec == "f64" else torch.float32
    phi = torch.empty(numel, dtype=odt, device=dev)
    psi = torch.empty(numel, dtype=odt, device=dev)
    ws = plan.workspace(dev)
    B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
    evs = ev.create(2 * reps)
    for r in range(reps):
        B.corr2d_set_timing_events(evs[2 * r], evs[2 * r + 1])
        B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
    torch.cuda.synchronize()
    ms = [ev.elapsed_ms(evs[2 * r], evs[2 * r + 1]) for r in range(reps)]
    B.corr2d_set_timing_events(None, None)
    ev.destroy(evs)
    del phi, psi, ws, plan, y
    torch.cuda.empty_cache()
    return float(np.median(ms))


def main(argv=None):
    ap = argparse.ArgumentParser(description="tile-shape autotuner of the correlation kernel")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--precs", default=",".join(CANDIDATES))
    args = ap.parse_args(argv)

    import torch

    from . import binding as B
    from .timing import HipEvents

    assert torch.cuda.is_available(), "the tuner times kernels on the GPU"
    B.lib()
    ev = HipEvents()
    timings = {}
    t0 = time.time()
    for prec in args.precs.split(","):
        for mc in M_CLASSES:
            for nc in N_CLASSES:
                res = {}
                for tile in CANDIDATES[prec]:
                    res[tile] = time_tile(B, torch, prec, mc, nc, tile, ev)
                timings[(prec, mc, nc)] = res
                print(f"{prec:11s} m={mc:4d} n={nc:6d} " +
                      " ".join(f"tile{t}={v:.4f}ms" for t, v in res.items()), flush=True)
    lines = rules_from_timings(timings)
    dev = torch.cuda.get_device_properties(0)
    write_table(lines, args.out, [f"written by paper_1808_00685_amd.tune on {dev.name} "
                                  f"({getattr(dev, 'gcnArchName', '')}) in {time.time() - t0:.0f} s",
                                  "size classes: m in " + str(M_CLASSES) + ", n in " + str(N_CLASSES)])
    print(f"wrote {len(lines)} rules to {args.out}", flush=True)


if __name__ == "__main__":
    main()
