"""Parity at the full workload sizes, in the launch configuration the
benchmark times: every entry of the full Phi and Psi against the oracle
(computed in row blocks), for the m=256 x n=16384 homocorrelation, the
m=128, 8192 x 2048 heterocorrelation and the batch of 256 data sets (the
persistent launch replayed from a hipGraph, against sequential launches and
the oracle).
"""
import numpy as np
import pytest

import oracle
from paper_1808_00685_amd import binding as B
from paper_1808_00685_amd import synth

from .gpu_helpers import (BF16_BAND_TOL, ELEMENT_TAU, TOL, aligned_rows, homo_full_error,
                          oracle_upper_blocks, packed_index, packed_rows, rel_fro)
from .lag_pairs import lag_sign_pairs

pytestmark = pytest.mark.gpu


def _sample_pairs(n, count, seed, centers=()):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    i, j = np.minimum(i, j), np.maximum(i, j)
    c = np.asarray(sorted(set(int(x) for x in centers if 0 <= x < n)), dtype=np.int64)
    if len(c):
        ci, cj = np.meshgrid(c, c, indexing="ij")
        keep = ci <= cj
        i = np.concatenate([i, ci[keep]])
        j = np.concatenate([j, cj[keep]])
    edge = np.array([0, n - 1, n // 2], dtype=np.int64)
    i = np.concatenate([i, edge, [0, 0, n - 2]])
    j = np.concatenate([j, edge, [n - 1, 1, n - 1]])
    return i.astype(np.int64), j.astype(np.int64)


@pytest.fixture(scope="module")
def large():
    import torch
    S, meta = synth.workload_large()
    return S, oracle_upper_blocks(oracle, S, torch.device("cuda:0"))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,basis,tol,flags,layout", [
    ("split_bf16", "auto", TOL["split_bf16"], 0, "upper_aligned"),
    ("split_f16", "auto", TOL["split_f16"], 0, "upper_aligned"),
    ("f32", "auto", TOL["f32"], 0, "upper_aligned"),
    ("split_bf16", "fourier", TOL["split_bf16"], 0, "upper_aligned"),
    ("split_bf16", "fourier", TOL["split_bf16"], B.FLAG_TRANSFORM_MATMUL, "upper_packed"),
    ("f32", "fourier", TOL["f32"], 0, "upper_aligned"),
    ("split_f16", "fourier", TOL["split_f16"], 0, "upper_aligned"),
    ("split_f16", "fourier", TOL["split_f16"], B.FLAG_SPLIT_ROWS, "upper_aligned"),
    ("split_bf16", "fourier", TOL["split_bf16"], B.FLAG_SPLIT_ROWS, "upper_aligned"),
    ("bf16", "auto", BF16_BAND_TOL, 0, "upper_aligned"),
    ("bf16", "fourier", TOL["bf16"], 0, "upper_aligned"),
])
def test_large_homo_full(gpu, large, prec, basis, tol, flags, layout):
    """m=256, n=16384 band workload, upper triangle stored (the bench's
    launch: the default, time basis), in both bases, through the radix FFT
    transform (the default at this m) and,
    forced by the flag, the table product: every entry of the full Phi and
    Psi against the oracle (relative Frobenius error over the full matrix,
    and each entry within its own bound, gpu_helpers.ELEMENT_TAU).  Plain
    BF16 meets the 2e-3 target in its default (time) basis; in the Fourier
    basis (1.9e-3 / 2.5e-3 measured) it is held to the format's derived bound."""
    import torch
    S, blocks = large
    n = S.shape[1]
    phi, psi, plan, ws = B.homo(torch.as_tensor(S, device=gpu), prec=prec, basis=basis,
                                layout=layout, flags=flags)
    torch.cuda.synchronize()
    rowsel = bool(flags & B.FLAG_SPLIT_ROWS)
    assert B.corr2d_plan_get_info(plan.handle).transform == (0 if flags & B.FLAG_TRANSFORM_MATMUL else 1)
    rows = aligned_rows if layout == "upper_aligned" else packed_rows
    planes = (phi, psi)
    # the row-selective split leaves chosen rows to hi*hi: no per-element bound
    fe = homo_full_error(blocks, lambda k, r0, r1: rows(planes[k], n, r0, r1),
                         tau=None if rowsel else ELEMENT_TAU[prec])
    if rowsel:
        nsel, order = B.selection(ws, plan)
        print(f"large {prec} row-selective: {nsel} of {len(order)} K blocks carry the low plane")
    e_phi, e_psi = fe.rel(0), fe.rel(1)
    print(f"large {prec}/{basis}/flags={flags}/{layout}: full-matrix rel.err phi={e_phi:.3e} "
          f"psi={e_psi:.3e} (largest error/bound {fe.bound_ratio:.3f})")
    assert fe.entries == n * (n + 1) // 2
    assert e_phi <= tol and e_psi <= tol
    assert fe.bound_ratio <= 1.0
    ii = np.arange(n)
    d = packed_index(ii, ii, n) if layout == "upper_packed" else B.upper_aligned_index(ii, ii, n)
    assert torch.all(psi[torch.as_tensor(d, device=gpu)] == 0)
    del phi, psi, ws


def test_large_upper_aligned_equals_packed(gpu, large):
    """The bench's launch in both upper layouts at m=256, n=16384: every
    aligned-layout entry equals the packed one bit for bit (so the sampled
    oracle check above covers both), and exactly the padding slots stay
    unwritten."""
    import torch
    S = large[0]
    m, n = S.shape
    y = torch.as_tensor(S, device=gpu)
    outs = {}
    for layout in ("upper_packed", "upper_aligned"):
        plan = B.Plan(m=m, n1=n, n2=0, prec="split_bf16", out_layout=layout, in_dtype="f64",
                      out_dtype="f32")
        numel = B.out_elements(layout, n)
        phi = torch.full((numel,), float("nan"), dtype=torch.float32, device=gpu)
        psi = torch.full((numel,), float("nan"), dtype=torch.float32, device=gpu)
        ws = plan.workspace(gpu)
        B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
        torch.cuda.synchronize()
        outs[layout] = (phi, psi)
        del ws, plan
    # packed order -> aligned slots, from the layout's definition (row starts
    # are cumulative row lengths N32 - 32 floor(i/32))
    ii = torch.arange(n, device=gpu, dtype=torch.int64)
    first = 32 * (ii // 32)
    alen = (n + 31) // 32 * 32 - first
    astart = torch.cumsum(alen, 0) - alen
    plen = n - ii
    rows = torch.repeat_interleave(ii, plen)
    pstart = torch.cumsum(plen, 0) - plen
    cols = torch.arange(rows.numel(), device=gpu, dtype=torch.int64) - pstart[rows] + rows
    aidx = astart[rows] + cols - first[rows]
    del cols
    for k in range(2):
        pk, al = outs["upper_packed"][k], outs["upper_aligned"][k]
        assert not torch.isnan(pk).any()
        assert torch.equal(al[aidx], pk)
        assert int(torch.isnan(al).sum()) == al.numel() - n * (n + 1) // 2
    del outs, aidx, rows


@pytest.fixture(scope="module")
def hetero_data():
    S1, S2, meta = synth.workload_hetero()
    Y1, Y2 = oracle.dynamic(S1)[0], oracle.dynamic(S2)[0]
    phi_o, psi_o = oracle.corr_ht(Y1, Y2)
    c1 = np.round(meta["set1"]["centers"]).astype(int)
    c2 = np.round(meta["set2"]["centers"]).astype(int)
    norms = (np.linalg.norm(Y1, axis=0), np.linalg.norm(Y2, axis=0),
             np.linalg.norm(oracle.noda_transform(Y2), axis=0))
    return S1, S2, meta, phi_o, psi_o, c1, c2, norms


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["f16", "fp8_e4m3", "split_bf16", "split_f16"])
def test_hetero_workload_full(gpu, hetero_data, prec):
    """m=128, 8192 x 2048 heterocorrelation with per-band scaling: every
    entry against the oracle."""
    import torch
    S1, S2, meta, phi_o, psi_o, c1, c2, (ny1, ny2, nz2) = hetero_data
    phi, psi, plan, ws = B.hetero(torch.as_tensor(S1, device=gpu), torch.as_tensor(S2, device=gpu),
                                  prec=prec)
    if prec in ("f16", "fp8_e4m3"):
        assert plan.info.per_band_scale == 1
    g_phi = phi.double().cpu().numpy()
    g_psi = psi.double().cpu().numpy()
    e_phi, e_psi = rel_fro(g_phi, phi_o), rel_fro(g_psi, psi_o)
    print(f"hetero {prec}: full-matrix rel.err phi={e_phi:.3e} psi={e_psi:.3e}")
    assert e_phi <= TOL[prec] and e_psi <= TOL[prec]
    # every entry within its own bound (gpu_helpers.ELEMENT_TAU)
    m, tau = S1.shape[0], ELEMENT_TAU[prec]
    assert np.all(np.abs(g_phi - phi_o) <= tau * np.outer(ny1, ny2) / (m - 1))
    assert np.all(np.abs(g_psi - psi_o) <= tau * np.outer(ny1, nz2) / (m - 1))
    # sign of Psi at band-centre pairs agrees with the oracle where it is not tiny
    cq, cg = psi_o[np.ix_(c1, c2)], g_psi[np.ix_(c1, c2)]
    big = np.abs(cq) > 0.05 * np.abs(cq).max()
    assert np.all(np.sign(cg[big]) == np.sign(cq[big]))
    # and with the generator's driver lags where those fix it
    li, lj, expected = lag_sign_pairs(meta)
    assert np.all(np.sign(g_psi[li, lj]) == expected)
    del phi, psi, ws


def _batch(count, seed, n_range):
    items = synth.batch_spec(count=count, seed=seed, n_range=n_range)
    data = [synth.batch_item_data(it) for it in items]
    return items, data


def _run_batched(gpu, items, data, prec, flags, layout="upper_packed"):
    import torch
    offs, ooffs, cur, ocur = [], [], 0, 0
    for it in items:
        offs.append(cur)
        ooffs.append(ocur)
        cur += it.m * it.n
        ocur += it.n * (it.n + 1) // 2 if layout == "upper_packed" else it.n * it.n
    y = torch.empty(cur, dtype=torch.float64, device=gpu)
    for it, S, o in zip(items, data, offs):
        y[o:o + it.m * it.n] = torch.as_tensor(S.ravel(), device=gpu)
    d = B.corr2d_desc_init(prec=prec, out_layout=layout, flags=flags)
    plan = B.Plan(d, items=[(it.m, it.n, o, 0, oo) for it, o, oo in zip(items, offs, ooffs)])
    phi = torch.zeros(ocur, dtype=torch.float32, device=gpu)
    psi = torch.zeros(ocur, dtype=torch.float32, device=gpu)
    ws = plan.workspace(gpu)
    return plan, y, phi, psi, ws, ooffs


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_batched_graph_matches_sequential_and_oracle(gpu, prec):
    import torch
    items, data = _batch(24, 77, (256, 1500))
    plan, y, phi, psi, ws, ooffs = _run_batched(gpu, items, data, prec, 0)
    B.corr2d_batched(plan.handle, y, phi, psi, ws)
    torch.cuda.synchronize()
    ref_phi, ref_psi = phi.clone(), psi.clone()
    # graph replays with eager work and synchronizations in between
    for rep in range(3):
        phi.zero_()
        psi.fill_(3.0)
        junk = torch.randn(1 << 20, device=gpu).sum()
        torch.cuda.synchronize()
        B.corr2d_batched(plan.handle, y, phi, psi, ws)
        torch.cuda.synchronize()
        assert torch.equal(phi, ref_phi) and torch.equal(psi, ref_psi), rep
        del junk
    # sequential launches (no persistent kernel, no graph) give the same values
    seq, ys, sphi, spsi, sws, _ = _run_batched(gpu, items, data, prec, B.FLAG_SEQUENTIAL)
    B.corr2d_batched(seq.handle, ys, sphi, spsi, sws)
    torch.cuda.synchronize()
    assert torch.equal(sphi, ref_phi) and torch.equal(spsi, ref_psi)
    # every data set against the oracle on sampled entries
    gp, gq = ref_phi.double().cpu().numpy(), ref_psi.double().cpu().numpy()
    for k, (it, S, oo) in enumerate(zip(items, data, ooffs)):
        i, j = _sample_pairs(it.n, 300, k)
        po, qo = oracle.corr2d_entries(S, i, j)
        pidx = oo + packed_index(i, j, it.n)
        assert rel_fro(gp[pidx], po) <= TOL[prec], k
        assert rel_fro(gq[pidx], qo) <= TOL[prec], k
        # and every sampled entry within its own bound (gpu_helpers.ELEMENT_TAU)
        Y, _ = oracle.dynamic(S)
        ny = np.linalg.norm(Y, axis=0)
        nz = np.linalg.norm(oracle.noda_transform(Y), axis=0)
        tau = ELEMENT_TAU[prec]
        assert np.all(np.abs(gp[pidx] - po) <= tau * ny[i] * ny[j] / (it.m - 1)), k
        assert np.all(np.abs(gq[pidx] - qo) <= tau * ny[i] * nz[j] / (it.m - 1)), k


@pytest.mark.timeout(1200)
def test_batched_full_size_every_set(gpu):
    """The batch of 256 data sets at its real size (m in 8..200, n in
    256..8192; the bench's launch): the graph-replayed persistent launch in
    FP32, split-FP16 and split-BF16, every data set's full Phi and Psi
    against the oracle, every entry within its own bound; FP32 sequential
    launches give the same bits.  FP32, split-FP16 and split-BF16 hold 1e-5
    (relative Frobenius over each full matrix) on every data set in the
    default time basis (split-BF16's worst, a data set whose Psi cancels
    about twentyfold, measures 9.1e-6; in the Fourier basis, where the
    rounding errors of its 8-bit halves pile up in the few rows that carry
    the bands, 5.4e-5)."""
    import time as _time
    import torch
    items = synth.batch_spec()
    data = [synth.batch_item_data(it) for it in items]
    outs = {}
    for name, prec, flags in (("graph", "f32", 0), ("split", "split_f16", 0),
                              ("split_bf16", "split_bf16", 0),
                              ("sequential", "f32", B.FLAG_SEQUENTIAL)):
        plan, y, phi, psi, ws, ooffs = _run_batched(gpu, items, data, prec, flags)
        B.corr2d_batched(plan.handle, y, phi, psi, ws)
        torch.cuda.synchronize()
        outs[name] = (phi, psi)
        del plan, ws, y
    assert torch.equal(outs["graph"][0], outs["sequential"][0])
    assert torch.equal(outs["graph"][1], outs["sequential"][1])
    del outs["sequential"]
    worst = {}
    total = {name: [0.0, 0.0, 0.0, 0.0] for name in outs}
    t0 = _time.time()
    for k, (it, S, oo) in enumerate(zip(items, data, ooffs)):
        blocks = oracle_upper_blocks(oracle, S, gpu)
        for name, prec in (("graph", "f32"), ("split", "split_f16"), ("split_bf16", "split_bf16")):
            planes = outs[name]
            fe = homo_full_error(blocks, lambda q, r0, r1: packed_rows(planes[q], it.n, r0, r1, oo),
                                 tau=ELEMENT_TAU[prec])
            assert fe.entries == it.n * (it.n + 1) // 2
            e = (fe.rel(0), fe.rel(1), fe.bound_ratio)
            for q in range(2):
                total[name][2 * q] += fe.num[q]
                total[name][2 * q + 1] += fe.den[q]
            if name not in worst or max(e[:2]) > max(worst[name][1][:2]):
                worst[name] = (k, e)
            assert e[0] <= TOL[prec] and e[1] <= TOL[prec], (name, k, it.m, it.n, e)
            assert e[2] <= 1.0, (name, k, it.m, it.n, e)
        del blocks
        if k % 32 == 31:
            print(f"batch: {k + 1} sets compared ({_time.time() - t0:.0f} s)", flush=True)
    for name, (k, e) in worst.items():
        t = total[name]
        print(f"batch {name}: whole batch rel.err phi={np.sqrt(t[0] / t[1]):.3e} "
              f"psi={np.sqrt(t[2] / t[3]):.3e}; worst set {k} (m={items[k].m}, n={items[k].n}) "
              f"phi={e[0]:.3e} psi={e[1]:.3e}, largest error/bound {e[2]:.3f}")
    t = total["split_bf16"]
    assert np.sqrt(t[0] / t[1]) <= TOL["split_bf16"] and np.sqrt(t[2] / t[3]) <= TOL["split_bf16"]


def test_batched_full_layout_and_no_graph(gpu):
    import torch
    items, data = _batch(6, 78, (256, 700))
    plan, y, phi, psi, ws, ooffs = _run_batched(gpu, items, data, "f64", B.FLAG_NO_GRAPH,
                                                layout="full")
    B.corr2d_batched(plan.handle, y, phi, psi, ws)
    torch.cuda.synchronize()
    gp, gq = phi.double().cpu().numpy(), psi.double().cpu().numpy()
    for it, S, oo in zip(items, data, ooffs):
        po, qo = oracle.corr2d(S)
        P = gp[oo:oo + it.n * it.n].reshape(it.n, it.n)
        Q = gq[oo:oo + it.n * it.n].reshape(it.n, it.n)
        # the output buffers are FP32 here: FP32 rounding bounds the error
        assert rel_fro(P, po) <= 1e-6 and rel_fro(Q, qo) <= 1e-6
        assert np.array_equal(P, P.T) and np.array_equal(Q, -Q.T)
