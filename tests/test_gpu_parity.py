"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every test runs the library's kernels on the GPU and compares element by
element with the oracle on the same seeded inputs, at the tolerances in
gpu_helpers.TOL.  Small cases cover several tiles and ragged tails; the large
workloads are checked on sampled entries the oracle computes one by one.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1808_00685_amd import binding as B
from paper_1808_00685_amd import synth

from .gpu_helpers import (ELEMENT_TAU, TOL, check_homo_structure, packed_index, rel_fro,
                          unpack_upper, unpack_upper_aligned)

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "split_bf16", "bf16", "f16", "fp8_e4m3", "split_f16"]


def _t(a, dev, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device=dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _rand(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n)) + 3.0


def _homo(S, dev, **kw):
    phi, psi, plan, ws = B.homo(_t(S, dev), **kw)
    return _np(phi), _np(psi), plan


# --------------------------------------------------------------------------
# Small and ragged cases, every precision
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n", [(2, 1), (3, 7), (11, 512), (17, 129), (33, 300), (64, 257)])
def test_homo_parity_small(gpu, prec, m, n):
    S = _rand(m, n, 1000 * m + n)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo(S, gpu, prec=prec)
    check_homo_structure(phi, psi)
    tol = TOL[prec]
    assert rel_fro(phi, phi_o) <= tol
    if m > 2:
        assert rel_fro(psi, psi_o) <= tol
    else:  # m = 2: Psi is identically zero
        assert np.abs(psi).max() <= 1e-6 * np.abs(phi).max()


def test_small_workload_f64(gpu):
    """The 11 x 512 four-band workload in FP64 (full 512 x 512 outputs)."""
    S, _ = synth.workload_small()
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo(S, gpu, prec="f64")
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= 1e-12
    assert rel_fro(psi, psi_o) <= 1e-12
    assert np.abs(np.diag(phi) - np.var(S, axis=0, ddof=1)).max() <= 1e-12 * np.abs(phi).max()


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "split_f16"])
@pytest.mark.parametrize("basis", ["fourier", "time"])
@pytest.mark.parametrize("hilbert", ["noda", "circular"])
def test_modes(gpu, prec, basis, hilbert):
    m, n = 24, 200
    S = _rand(m, n, 7)
    phi_o, psi_o = oracle.corr2d(S, hilbert=hilbert)
    phi, psi, _ = _homo(S, gpu, prec=prec, basis=basis, hilbert=hilbert)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]


@pytest.mark.parametrize("norm,val", [("paper", 0.0), ("custom", 0.37)])
def test_norm_modes(gpu, norm, val):
    m, n = 13, 150
    S = _rand(m, n, 8)
    phi_o, psi_o = oracle.corr2d(S, norm=norm, norm_value=val)
    phi, psi, _ = _homo(S, gpu, prec="f64", norm=norm, norm_value=val)
    assert rel_fro(phi, phi_o) <= 1e-12 and rel_fro(psi, psi_o) <= 1e-12


def test_user_reference_and_f32_input_and_strides(gpu):
    import torch
    m, n, ld = 20, 150, 170
    S = _rand(m, n, 9)
    ref = S[0] + 0.25
    phi_o, psi_o = oracle.corr2d(S, ref1=ref)
    big = np.zeros((m, ld))
    big[:, :n] = S
    y = _t(big, gpu)[:, :n]
    phi, psi, _, _ = B.homo(y, ref=_t(ref, gpu), prec="f64")
    assert rel_fro(_np(phi), phi_o) <= 1e-12 and rel_fro(_np(psi), psi_o) <= 1e-12
    # FP32 input (the FP64 mean of the FP32 values)
    S32 = S.astype(np.float32)
    phi_o, psi_o = oracle.corr2d(S32.astype(np.float64))
    phi, psi, _, _ = B.homo(_t(S32, gpu, torch.float32), prec="f32")
    assert rel_fro(_np(phi), phi_o) <= 1e-5 and rel_fro(_np(psi), psi_o) <= 1e-5


def test_f64_output_of_reduced_precision_and_full_ld_out(gpu):
    import torch
    m, n, ldo = 16, 140, 160
    S = _rand(m, n, 10)
    phi_o, psi_o = oracle.corr2d(S)
    d = B.corr2d_desc_init(m=m, n1=n, prec="f32", out_dtype="f64", ld_out=ldo)
    plan = B.Plan(d)
    phi = torch.full((n, ldo), 7.0, dtype=torch.float64, device=gpu)
    psi = torch.full((n, ldo), 7.0, dtype=torch.float64, device=gpu)
    ws = plan.workspace(gpu)
    B.corr2d_homo(plan.handle, _t(S, gpu), None, phi, psi, ws)
    ph, ps = _np(phi), _np(psi)
    assert np.all(ph[:, n:] == 7.0) and np.all(ps[:, n:] == 7.0)   # padding columns untouched
    assert rel_fro(ph[:, :n], phi_o) <= 1e-5 and rel_fro(ps[:, :n], psi_o) <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "split_bf16"])
def test_upper_packed_layout(gpu, prec):
    m, n = 21, 333
    S = _rand(m, n, 11)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo(S, gpu, prec=prec, layout="upper_packed")
    assert phi.shape == (n * (n + 1) // 2,)
    P, Q = unpack_upper(phi, n), unpack_upper(psi, n)
    iu = np.triu_indices(n)
    assert rel_fro(P[iu], phi_o[iu]) <= TOL[prec]
    assert rel_fro(Q[iu], psi_o[iu]) <= TOL[prec]
    assert np.all(np.diag(Q) == 0)


def _homo_nan_filled(S, dev, **kw):
    """Homocorrelation into NaN-filled outputs (to see which slots are written)."""
    import torch
    m, n = S.shape
    prec = kw.get("prec", "split_bf16")
    out = "f64" if prec == "f64" else "f32"
    plan = B.Plan(m=m, n1=n, n2=0, in_dtype="f64", out_dtype=out, **kw)
    numel = B.out_elements(B.LAYOUT_NAMES[plan.desc.out_layout], n)
    tdt = torch.float64 if out == "f64" else torch.float32
    phi = torch.full((numel,), float("nan"), dtype=tdt, device=dev)
    psi = torch.full((numel,), float("nan"), dtype=tdt, device=dev)
    ws = plan.workspace(dev)
    B.corr2d_homo(plan.handle, _t(S, dev), None, phi, psi, ws)
    return _np(phi), _np(psi), plan


@pytest.mark.parametrize("prec,tile", [("f64", 1), ("f64", 2), ("f32", 1), ("f32", 2), ("fp8_e4m3", 1),
                                       ("fp8_e4m3", 2), ("split_bf16", 2), ("split_bf16", 3),
                                       ("bf16", 3), ("f16", 2)])
@pytest.mark.parametrize("n", [1, 33, 333])
def test_upper_aligned_layout(gpu, prec, tile, n):
    # every kernel family writes the row-aligned triangle: entries j >= i at
    # the layout's offsets, padding slots untouched
    m = 21
    S = _rand(m, n, 12 + n)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo_nan_filled(S, gpu, prec=prec, tile=tile, out_layout="upper_aligned")
    assert phi.shape == (B.upper_aligned_elements(n),)
    P, pad = unpack_upper_aligned(phi, n)
    Q, _ = unpack_upper_aligned(psi, n)
    assert np.all(np.isnan(phi[pad])) and np.all(np.isnan(psi[pad]))
    assert not np.any(np.isnan(phi[~pad])) and not np.any(np.isnan(psi[~pad]))
    iu = np.triu_indices(n)
    assert rel_fro(P[iu], phi_o[iu]) <= TOL[prec]
    if n > 1:
        assert rel_fro(Q[iu], psi_o[iu]) <= TOL[prec]
    assert np.all(np.diag(Q) == 0)


def test_upper_aligned_equals_packed_bitwise(gpu):
    # the layouts differ only in addressing: the same plan settings give the
    # same values in both
    m, n = 64, 1500
    S = _rand(m, n, 21)
    for prec in ("split_bf16", "f32"):
        pa, qa, _ = _homo_nan_filled(S, gpu, prec=prec, out_layout="upper_aligned")
        pp, qp, _ = _homo_nan_filled(S, gpu, prec=prec, out_layout="upper_packed")
        A, _ = unpack_upper_aligned(pa, n)
        iu = np.triu_indices(n)
        assert np.array_equal(A[iu], unpack_upper(pp, n)[iu])
        A, _ = unpack_upper_aligned(qa, n)
        assert np.array_equal(A[iu], unpack_upper(qp, n)[iu])


@pytest.mark.parametrize("prec", ["f32", "split_bf16", "bf16"])
def test_batched_upper_aligned(gpu, prec):
    # batched sets written in the aligned layout at their own offsets; the
    # 700-point set has interior tiles (stored straight from the
    # accumulators by the persistent 16-bit kernel)
    import torch
    sets = [_rand(9, 70, 31), _rand(40, 333, 32), _rand(3, 32, 33), _rand(24, 700, 34)]
    items, ycat, oo, io = [], [], 0, 0
    for S in sets:
        m, n = S.shape
        items.append((m, n, io, 0, oo))
        ycat.append(S.ravel())
        io += m * n
        oo += B.upper_aligned_elements(n) + 5        # offsets need not be aligned
    plan = B.Plan(prec=prec, out_layout="upper_aligned", in_dtype="f64", out_dtype="f32",
                  items=items)
    assert plan.info.out_elements == items[-1][4] + B.upper_aligned_elements(sets[-1].shape[1])
    y = _t(np.concatenate(ycat), gpu)
    phi = torch.full((oo,), float("nan"), dtype=torch.float32, device=gpu)
    psi = torch.full((oo,), float("nan"), dtype=torch.float32, device=gpu)
    ws = plan.workspace(gpu)
    B.corr2d_batched(plan.handle, y, phi, psi, ws)
    gp, gq = _np(phi), _np(psi)
    for S, it in zip(sets, items):
        n = S.shape[1]
        e = B.upper_aligned_elements(n)
        P, pad = unpack_upper_aligned(gp[it[4]:it[4] + e], n)
        Q, _ = unpack_upper_aligned(gq[it[4]:it[4] + e], n)
        phi_o, psi_o = oracle.corr2d(S)
        iu = np.triu_indices(n)
        assert rel_fro(P[iu], phi_o[iu]) <= TOL[prec]
        assert rel_fro(Q[iu], psi_o[iu]) <= TOL[prec]
        assert np.all(np.isnan(gp[it[4]:it[4] + e][pad]))
        assert np.all(np.diag(Q) == 0)


@pytest.mark.parametrize("prec", ["split_bf16", "bf16", "f16", "split_f16"])
@pytest.mark.parametrize("tile", [2, 3])
@pytest.mark.parametrize("layout", ["full", "upper_packed", "upper_aligned"])
def test_lds_staged_tile_shapes(gpu, prec, tile, layout):
    # both tile shapes of the LDS-staged kernel (256 x 128 and 128 x 128),
    # with ragged edges and several diagonal-crossing tiles
    m, n = 37, 700
    S = _rand(m, n, 77)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, plan = _homo(S, gpu, prec=prec, layout=layout, tile=tile)
    info = plan.info
    assert (info.tile_m, info.tile_n) == ((256, 128) if tile == 2 else (128, 128))
    if layout != "full":
        if layout == "upper_packed":
            phi, psi = unpack_upper(phi, n), unpack_upper(psi, n)
        else:
            phi, psi = unpack_upper_aligned(phi, n)[0], unpack_upper_aligned(psi, n)[0]
        iu = np.triu_indices(n)
        assert rel_fro(phi[iu], phi_o[iu]) <= TOL[prec]
        assert rel_fro(psi[iu], psi_o[iu]) <= TOL[prec]
        assert np.all(np.diag(psi) == 0)
    else:
        check_homo_structure(phi, psi)
        assert rel_fro(phi, phi_o) <= TOL[prec]
        assert rel_fro(psi, psi_o) <= TOL[prec]
    S2 = _rand(m, 300, 78)
    phi_o, psi_o = oracle.corr2d(S, S2)
    phi, psi, _, _ = B.hetero(_t(S, gpu), _t(S2, gpu), prec=prec, tile=tile)
    assert rel_fro(_np(phi), phi_o) <= TOL[prec]
    assert rel_fro(_np(psi), psi_o) <= TOL[prec]


@pytest.mark.parametrize("layout", ["full", "upper_packed", "upper_aligned"])
def test_f64_128x64_tile(gpu, layout):
    """FP64's tile 2 (128 x 64: row tiles twice as tall as column tiles) in
    every layout with ragged edges and diagonal-crossing tiles, and for a
    heterocorrelation; bit-identical to the 64 x 64 tile (each element sums
    its K terms in the same order)."""
    m, n = 37, 700
    S = _rand(m, n, 79)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, plan = _homo_nan_filled(S, gpu, prec="f64", tile=2, out_layout=layout)
    assert (plan.info.tile_m, plan.info.tile_n) == (128, 64)
    ref = _homo_nan_filled(S, gpu, prec="f64", tile=1, out_layout=layout)
    assert np.array_equal(np.nan_to_num(phi, nan=7.0), np.nan_to_num(ref[0], nan=7.0))
    assert np.array_equal(np.nan_to_num(psi, nan=7.0), np.nan_to_num(ref[1], nan=7.0))
    if layout == "full":
        P, Q = phi.reshape(n, n), psi.reshape(n, n)
    elif layout == "upper_packed":
        P, Q = unpack_upper(phi, n), unpack_upper(psi, n)
    else:
        P, Q = unpack_upper_aligned(phi, n)[0], unpack_upper_aligned(psi, n)[0]
    iu = np.triu_indices(n)
    assert rel_fro(P[iu], phi_o[iu]) <= TOL["f64"] and rel_fro(Q[iu], psi_o[iu]) <= TOL["f64"]
    S2 = _rand(m, 300, 80)
    phi_o, psi_o = oracle.corr2d(S, S2)
    phi, psi, _, _ = B.hetero(_t(S, gpu), _t(S2, gpu), prec="f64", tile=2)
    assert rel_fro(_np(phi), phi_o) <= TOL["f64"] and rel_fro(_np(psi), psi_o) <= TOL["f64"]


# --------------------------------------------------------------------------
# Heterocorrelation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n1,n2", [(5, 3, 200), (32, 300, 129), (40, 128, 128)])
def test_hetero_parity(gpu, prec, m, n1, n2):
    S1 = _rand(m, n1, 20 + m)
    S2 = _rand(m, n2, 30 + m)
    phi_o, psi_o = oracle.corr2d(S1, S2)
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec=prec)
    assert rel_fro(_np(phi), phi_o) <= TOL[prec]
    assert rel_fro(_np(psi), psi_o) <= TOL[prec]


@pytest.mark.parametrize("prec", ["split_bf16", "f32", "bf16", "f64", "f16", "fp8_e4m3", "split_f16"])
@pytest.mark.parametrize("m,n1,n2", [(256, 640, 0), (181, 500, 0), (128, 400, 300)])
def test_error_within_elementwise_bound(gpu, prec, m, n1, n2):
    """Every entry lies within its own bound, whatever its cancellation:
    with sum|a_k||b_k| <= ||a|| ||b|| and ||a_i|| = sqrt(m) ||y_i||
    (Parseval on the packed half spectrum), an operand or product error of
    relative size tau gives |err_ij| <= tau ||y_i|| ||(N y)_j|| / (m - 1)
    for Psi and the same with y_j for Phi (FFT transform at m = 256, table
    product at m = 181, a heterocorrelation)."""
    S1 = _rand(m, n1, 760 + m)
    S2 = _rand(m, n2, 761 + m) * 3.0 if n2 else None
    phi_o, psi_o = oracle.corr2d(S1, S2)
    if n2:
        phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec=prec)
    else:
        phi, psi, _, _ = B.homo(_t(S1, gpu), prec=prec)
    phi, psi = _np(phi), _np(psi)
    Y1, _ = oracle.dynamic(S1)
    Y2 = Y1 if S2 is None else oracle.dynamic(S2)[0]
    ny1 = np.linalg.norm(Y1, axis=0)
    ny2 = np.linalg.norm(Y2, axis=0)
    nz2 = np.linalg.norm(oracle.noda_transform(Y2), axis=0)
    tau = ELEMENT_TAU[prec]
    bound_phi = tau * np.outer(ny1, ny2) / (m - 1)
    bound_psi = tau * np.outer(ny1, nz2) / (m - 1)
    assert np.all(np.abs(phi - phi_o) <= bound_phi)
    assert np.all(np.abs(psi - psi_o) <= bound_psi)
    # the bound is not vacuous: typical entries lie above it (|cos| ~ 1/sqrt(m)
    # against tau)
    # (FP8's bound only catches gross errors)
    if tau <= 2.0 ** -6:
        assert np.median(np.abs(phi_o) / bound_phi) > (10.0 if tau <= 2.0 ** -9 else 1.5)


@pytest.mark.parametrize("prec", ["split_bf16", "bf16", "f16", "split_f16"])
def test_hetero_direct_and_staged_stores_agree(gpu, prec):
    """Interior tiles of a heterocorrelation are stored straight from the
    accumulators when every output row is whole 128-byte lines (row stride
    a multiple of 32, aligned output), else through LDS: the three calls
    below (aligned; output shifted by one element; row stride n2 + 1) give
    the same bits, and match the oracle."""
    import torch
    m, n1, n2 = 64, 384, 256
    S1, S2 = _rand(m, n1, 750), _rand(m, n2, 751)
    y1, y2 = _t(S1, gpu), _t(S2, gpu)
    got = []
    for shift, ld in ((0, n2), (1, n2), (0, n2 + 1)):
        plan = B.Plan(m=m, n1=n1, n2=n2, prec=prec, ld_out=ld)
        ws = plan.workspace(gpu)
        bufs = [torch.full((n1 * ld + shift,), float("nan"), dtype=torch.float32, device=gpu)
                for _ in range(2)]
        phi, psi = (b[shift:] for b in bufs)
        B.corr2d_hetero(plan.handle, y1, None, y2, None, phi, psi, ws)
        torch.cuda.synchronize()
        got.append(tuple(x.view(n1, ld)[:, :n2].cpu() for x in (phi, psi)))
    for g in got[1:]:
        assert torch.equal(g[0], got[0][0]) and torch.equal(g[1], got[0][1])
    phi_o, psi_o = oracle.corr2d(S1, S2)
    assert rel_fro(got[0][0].numpy(), phi_o) <= TOL[prec]
    assert rel_fro(got[0][1].numpy(), psi_o) <= TOL[prec]


def test_hetero_circular_and_refs(gpu):
    m, n1, n2 = 18, 90, 70
    S1, S2 = _rand(m, n1, 40), _rand(m, n2, 41)
    r1, r2 = S1[3] - 0.1, None
    phi_o, psi_o = oracle.corr2d(S1, S2, ref1=r1, hilbert="circular")
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), ref1=_t(r1, gpu), prec="f64",
                              hilbert="circular")
    assert rel_fro(_np(phi), phi_o) <= 1e-12 and rel_fro(_np(psi), psi_o) <= 1e-12


def test_hetero_of_same_set_equals_homo(gpu):
    m, n = 12, 300
    S = _rand(m, n, 50)
    ph, ps, _ = _homo(S, gpu, prec="f64")
    hph, hps, _, _ = B.hetero(_t(S, gpu), _t(S, gpu), prec="f64")
    hph, hps = _np(hph), _np(hps)
    iu = np.triu_indices(n)
    assert np.array_equal(ph[iu], hph[iu])
    assert np.array_equal(ps[iu][iu[0] != iu[1]], hps[iu][iu[0] != iu[1]])


# --------------------------------------------------------------------------
# Method-level properties on the GPU output
# --------------------------------------------------------------------------
def test_phase_lag_sign_on_gpu(gpu):
    m, n = 41, 256
    nu = np.arange(n)
    t = np.arange(m)[:, None]
    T = 1.5 * (m - 1)
    prof1 = 4.0 / ((nu - 60) ** 2 + 4.0)
    prof2 = 4.0 / ((nu - 190) ** 2 + 4.0)
    for ph1, ph2 in [(0.2, 1.4), (1.4, 0.2)]:
        S = ((1 + 0.5 * np.sin(2 * math.pi * t / T + ph1)) * prof1[None, :]
             + (1 + 0.5 * np.sin(2 * math.pi * t / T + ph2)) * prof2[None, :])
        _, psi, _ = _homo(S, gpu, prec="split_bf16")
        assert np.sign(psi[60, 190]) == np.sign(math.sin(ph1 - ph2))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16"])
@pytest.mark.parametrize("m", [32, 128])
def test_fig1_cases_on_gpu(gpu, prec, m):
    """The special cases of Fig. 1 (Sec. 2) through the GPU path (table
    product at m = 32, radix FFT at m = 128): variables with one response
    (amplitudes 1, 2.5, -0.5) correlate purely synchronously, Psi vanishing
    to within each entry's bound and Phi signed by Noda's rules 1 and 2; a
    quarter-period lag at a Fourier bin correlates purely asynchronously,
    Phi vanishing to within the bound and Psi > 0 for the leading one."""
    tau = ELEMENT_TAU[prec]

    def norms(S):
        Y, _ = oracle.dynamic(S)
        return np.linalg.norm(Y, axis=0), np.linalg.norm(oracle.noda_transform(Y), axis=0)

    base = _rand(m, 1, 4 + m)
    S = np.hstack([base, 2.5 * base, -0.5 * base])
    phi, psi, _ = _homo(S, gpu, prec=prec)
    ny, nz = norms(S)
    assert np.all(np.abs(psi) <= tau * np.outer(ny, nz) / (m - 1))
    assert phi[0, 1] > 0 and phi[0, 2] < 0 and phi[1, 2] < 0
    p = 3
    t = np.arange(m)[:, None]
    S = np.cos(2 * math.pi * p * t / m + np.array([math.pi / 2, 0.0])[None, :])
    phi, psi, _ = _homo(S, gpu, prec=prec)
    ny, nz = norms(S)
    assert abs(phi[0, 1]) <= tau * ny[0] * ny[1] / (m - 1)
    assert psi[0, 1] > 0.1 and psi[1, 0] < -0.1


def test_determinism(gpu):
    S = _rand(30, 500, 60)
    a = _homo(S, gpu, prec="split_bf16")
    b = _homo(S, gpu, prec="split_bf16")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# --------------------------------------------------------------------------
# Medium workload (m=64, n=4096), full comparison
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_medium_workload_full(gpu, prec):
    S, _ = synth.workload_medium()
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo(S, gpu, prec=prec)
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]


# --------------------------------------------------------------------------
# Result scaling (Pearson, Pareto, general alpha)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16", "fp8_e4m3"])
@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_scaling_parity(gpu, prec, alpha):
    m, n = 23, 300
    rng = np.random.default_rng(91)
    # bands of very different intensity: scaling evens them out
    S = _rand(m, n, 90) * rng.uniform(1e-3, 1e2, size=n)
    S[:, 7] = 2.0             # constant variable: sigma = 0, left unscaled
    phi_o, psi_o = oracle.corr2d(S, alpha=alpha)
    phi, psi, _ = _homo(S, gpu, prec=prec, alpha=alpha)
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]
    assert np.all(phi[7] == 0) and np.all(psi[:, 7] == 0)
    if alpha == 1.0 and prec in ("f64", "f32", "split_bf16"):
        d = np.diag(phi)
        assert np.all(np.abs(np.delete(d, 7) - 1.0) <= 10 * TOL[prec])


def test_scaling_hetero_ref_and_batched(gpu):
    import torch
    m, n1, n2 = 17, 200, 90
    S1, S2 = _rand(m, n1, 92), _rand(m, n2, 93) * 50.0
    r1 = S1[2] + 0.01
    phi_o, psi_o = oracle.corr2d(S1, S2, ref1=r1, alpha=0.7)
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), ref1=_t(r1, gpu), prec="split_bf16", alpha=0.7)
    assert rel_fro(_np(phi), phi_o) <= TOL["split_bf16"]
    assert rel_fro(_np(psi), psi_o) <= TOL["split_bf16"]
    # batched plan: every data set scaled with its own sigma
    sets = [_rand(11, 150, 94) * 3.0, _rand(40, 260, 95), _rand(8, 70, 96) * 0.01]
    offs, ooffs, cur, ocur = [], [], 0, 0
    for S in sets:
        offs.append(cur)
        ooffs.append(ocur)
        cur += S.size
        ocur += S.shape[1] * (S.shape[1] + 1) // 2
    y = torch.cat([_t(S, gpu).reshape(-1) for S in sets])
    d = B.corr2d_desc_init(prec="f32", out_layout="upper_packed", scale_alpha=1.0)
    plan = B.Plan(d, items=[(S.shape[0], S.shape[1], o, 0, oo) for S, o, oo in zip(sets, offs, ooffs)])
    ph = torch.zeros(ocur, dtype=torch.float32, device=gpu)
    ps = torch.zeros(ocur, dtype=torch.float32, device=gpu)
    ws = plan.workspace(gpu)
    B.corr2d_batched(plan.handle, y, ph, ps, ws)
    gp, gq = _np(ph), _np(ps)
    for S, oo in zip(sets, ooffs):
        n = S.shape[1]
        po, qo = oracle.corr2d(S, alpha=1.0)
        P = unpack_upper(gp[oo:oo + n * (n + 1) // 2], n)
        Q = unpack_upper(gq[oo:oo + n * (n + 1) // 2], n)
        iu = np.triu_indices(n)
        assert rel_fro(P[iu], po[iu]) <= TOL["f32"]
        assert rel_fro(Q[iu], qo[iu]) <= TOL["f32"]


# --------------------------------------------------------------------------
# The R code's bin list (Sec. 4.2) with the paper's norm
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16", "fp8_e4m3"])
@pytest.mark.parametrize("m", [2, 3, 16, 37])
def test_r_compat_parity(gpu, prec, m):
    n = 150
    S = _rand(m, n, 300 + m)
    phi_o, psi_o = oracle.corr2d(S, hilbert="r_compat", norm="paper")
    phi, psi, _ = _homo(S, gpu, prec=prec, hilbert="r_compat", norm="paper")
    if m == 2:   # only DC is kept, and it is zero after centring
        assert np.abs(phi).max() < 1e-6 and np.abs(psi).max() < 1e-6
        return
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]


def test_r_compat_hetero_and_scaled(gpu):
    m, n1, n2 = 24, 130, 70
    S1, S2 = _rand(m, n1, 310), _rand(m, n2, 311) * 4.0
    phi_o, psi_o = oracle.corr2d(S1, S2, hilbert="r_compat", norm="paper", alpha=0.5)
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec="split_bf16", hilbert="r_compat",
                              norm="paper", alpha=0.5)
    assert rel_fro(_np(phi), phi_o) <= TOL["split_bf16"]
    assert rel_fro(_np(psi), psi_o) <= TOL["split_bf16"]


# --------------------------------------------------------------------------
# Interpolation to equidistant perturbation values (Sec. 4.1)
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# The result object of Sec. 3: reference spectra, complex FT, spectral axes
# --------------------------------------------------------------------------
def _mean_tol(m, S):
    # an m-term FP64 sum in another order than the oracle's
    return 4 * m * 2.0 ** -52 * float(np.abs(S).max())


@pytest.mark.parametrize("prec,m,n,in32", [("f64", 11, 512, False), ("f32", 64, 300, True),
                                           ("split_bf16", 256, 129, False), ("fp8_e4m3", 128, 70, False),
                                           ("f64", 1024, 33, True), ("bf16", 2, 1, False)])
def test_reference_spectrum_is_the_mean(gpu, prec, m, n, in32):
    """The perturbation mean each call subtracts (Eq. (ref)), from the
    table-product path's centring kernel and from the FFT kernel's fused
    centring, equals the oracle's FP64 mean; ft is phi + i psi."""
    import torch
    S = _rand(m, n, 700 + m)
    if in32:
        S = S.astype(np.float32).astype(np.float64)
    y = _t(S, gpu, torch.float32 if in32 else torch.float64)
    r = B.corr2d(y, prec=prec)
    assert r.plan.info.transform == (1 if m in (128, 256, 1024) else 0)
    _, mean_o = oracle.dynamic(S)
    ref1 = _np(r.ref1)
    assert ref1.shape == (n,)
    assert np.abs(ref1 - mean_o).max() <= _mean_tol(m, S)
    assert r.ref2 is r.ref1
    assert torch.equal(r.ft.real, r.phi) and torch.equal(r.ft.imag, r.psi)
    assert np.array_equal(r.wave1.numpy(), np.arange(n)) and r.wave2 is r.wave1
    phi_o, psi_o = oracle.corr2d(S)
    assert rel_fro(_np(r.phi), phi_o) <= TOL[prec]
    assert rel_fro(_np(r.psi), psi_o) <= TOL[prec]


def test_fused_centring_single_call(gpu):
    """The centring fused into the table-product transform (m <= 256 and a
    launch of >= 512 workgroups: m = 200, n = 16384, two row tiles per 64
    spectral points) writes the oracle's FP64 mean (Eq. (ref)), and sampled
    entries of Phi and Psi (Eqs. (disHTsyn), (disHTasyn)) match the oracle's."""
    import torch
    m, n = 200, 16384
    S = _rand(m, n, 720)
    r = B.corr2d(_t(S, gpu), prec="split_f16", layout="upper_aligned")
    torch.cuda.synchronize()
    assert r.plan.info.transform == 0
    _, mean_o = oracle.dynamic(S)
    assert np.abs(_np(r.ref1) - mean_o).max() <= _mean_tol(m, S)
    rng = np.random.default_rng(721)
    i = rng.integers(0, n, 4000)
    j = rng.integers(0, n, 4000)
    i, j = np.minimum(i, j), np.maximum(i, j)
    i[:64], j[:64] = np.arange(64) * 255, n - 1 - np.arange(64)   # first and last column blocks
    idx = torch.as_tensor(B.upper_aligned_index(i, j, n), device=gpu)
    phi_o, psi_o = oracle.corr2d_entries(S, i, j)
    assert rel_fro(_np(r.phi[idx]), phi_o) <= TOL["split_f16"]
    assert rel_fro(_np(r.psi[idx]), psi_o) <= TOL["split_f16"]


@pytest.mark.parametrize("m", [32, 256])
def test_reference_spectra_hetero_given_and_mean(gpu, m):
    """Heterocorrelation with a caller's ref1 and the mean for set 2: Ref1
    is the caller's spectrum bit for bit, Ref2 the mean of y2; the spectral
    axes are passed through."""
    import torch
    n1, n2 = 150, 90
    S1, S2 = _rand(m, n1, 710), _rand(m, n2, 711) * 5.0
    r1 = S1[3] - 0.25
    w1 = torch.linspace(1600.0, 1500.0, n1, dtype=torch.float64)
    r = B.corr2d(_t(S1, gpu), _t(S2, gpu), ref1=_t(r1, gpu), wave1=w1, prec="f32")
    assert np.array_equal(_np(r.ref1), r1)
    _, mean2 = oracle.dynamic(S2)
    assert np.abs(_np(r.ref2) - mean2).max() <= _mean_tol(m, S2)
    assert r.wave1 is w1 and np.array_equal(r.wave2.numpy(), np.arange(n2))
    phi_o, psi_o = oracle.corr2d(S1, S2, ref1=r1)
    assert rel_fro(_np(r.phi), phi_o) <= TOL["f32"]
    assert rel_fro(_np(r.psi), psi_o) <= TOL["f32"]
    assert tuple(r.ft.shape) == (n1, n2)


@pytest.mark.parametrize("m_out", [40, 128])
def test_reference_spectrum_after_interpolation(gpu, m_out):
    """With interpolation the mean is taken over the resampled spectra."""
    m_in, n = 23, 140
    t = _uneven(m_in, 720)
    S = _rand(m_in, n, 721)
    Si = oracle.interpolate(S, t, m_out, "spline")
    r = B.corr2d(_t(S, gpu), prec="split_bf16", interp="spline", t_in=t, m_out=m_out)
    _, mean_o = oracle.dynamic(Si)
    assert np.abs(_np(r.ref1) - mean_o).max() <= 1e-12 * float(np.abs(Si).max())


def test_reference_spectrum_follows_each_call(gpu):
    """A second call on the same plan and workspace rewrites the reference."""
    import torch
    m, n = 64, 200
    S1, S2 = _rand(m, n, 730), _rand(m, n, 731) - 7.0
    plan = B.Plan(m=m, n1=n, prec="f32")
    ws = plan.workspace(gpu)
    phi = torch.empty(n * n, dtype=torch.float32, device=gpu)
    psi = torch.empty_like(phi)
    for S in (S1, S2):
        B.corr2d_homo(plan.handle, _t(S, gpu), None, phi, psi, ws)
        got = _np(B.workspace_vector(ws, plan.info.ref1_offset, n))
        assert np.abs(got - oracle.dynamic(S)[1]).max() <= _mean_tol(m, S)


def test_corr2d_bundle_rejects_mixed_arguments(gpu):
    y = _t(_rand(8, 10, 740), gpu)
    with pytest.raises(ValueError):
        B.corr2d(y, ref2=y[0])
    with pytest.raises(ValueError):
        B.corr2d(y, y, layout="upper_packed")
    with pytest.raises(ValueError):
        B.hetero(y, _t(_rand(9, 10, 741), gpu))


def _uneven(m_in, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.uniform(0.3, 2.5, size=m_in))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16"])
@pytest.mark.parametrize("method", ["linear", "spline"])
@pytest.mark.parametrize("m_in,m_out", [(20, 32), (2, 9), (3, 8), (70, 64)])
def test_interpolation_parity(gpu, prec, method, m_in, m_out):
    n = 210
    t = _uneven(m_in, 400 + m_in)
    S = _rand(m_in, n, 401 + m_in)
    Si = oracle.interpolate(S, t, m_out, method)
    phi_o, psi_o = oracle.corr2d(Si)
    phi, psi, plan = _homo(S, gpu, prec=prec, interp=method, t_in=t, m_out=m_out)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    if m_in == 2:
        # two input rows: every resampled column follows the same straight
        # line in t, so Psi = b_i b_j x^T N x vanishes (N antisymmetric)
        assert np.abs(psi_o).max() <= 1e-14 * np.abs(phi_o).max()
        assert np.abs(psi).max() <= TOL[prec] * np.abs(phi).max()
    else:
        assert rel_fro(psi, psi_o) <= TOL[prec]


def test_interpolation_hetero_f32_input_scaled(gpu):
    import torch
    m_in, m_out = 15, 40
    t = _uneven(m_in, 410)
    S1, S2 = _rand(m_in, 120, 411), _rand(m_in, 90, 412) * 7.0
    S1i, S2i = oracle.interpolate(S1, t, m_out, "spline"), oracle.interpolate(S2, t, m_out, "spline")
    phi_o, psi_o = oracle.corr2d(S1i, S2i, alpha=0.5)
    y1 = _t(S1, gpu, torch.float32)
    y2 = _t(S2, gpu, torch.float32)
    # FP32 input: compare with the oracle on the same FP32-rounded spectra
    S1f, S2f = S1.astype(np.float32).astype(np.float64), S2.astype(np.float32).astype(np.float64)
    phi_o, psi_o = oracle.corr2d(oracle.interpolate(S1f, t, m_out, "spline"),
                                 oracle.interpolate(S2f, t, m_out, "spline"), alpha=0.5)
    phi, psi, _, _ = B.hetero(y1, y2, prec="f64", interp="spline", t_in=t, m_out=m_out, alpha=0.5)
    assert rel_fro(_np(phi), phi_o) <= 1e-12
    assert rel_fro(_np(psi), psi_o) <= 1e-12


# --------------------------------------------------------------------------
# Radix FFT transform (power-of-two 128 <= m <= 1024, Fourier basis)
# --------------------------------------------------------------------------
FFT_PRECS = ["f64", "f32", "split_bf16", "bf16", "f16", "fp8_e4m3", "split_f16"]


def _transform(plan):
    return B.corr2d_plan_get_info(plan.handle).transform


@pytest.mark.parametrize("basis", ["fourier", "time"])
@pytest.mark.parametrize("prec", FFT_PRECS)
@pytest.mark.parametrize("m,n", [(128, 300), (256, 129), (512, 70), (1024, 33)])
def test_fft_transform_parity(gpu, prec, m, n, basis):
    """Every FFT length (L = 256 .. 2048: radix 8 passes with a radix-4 or
    radix-2 last pass), operand format and basis; ragged n leaves padded
    points."""
    S = _rand(m, n, 31 * m + n)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, plan = _homo(S, gpu, prec=prec, basis=basis)
    assert _transform(plan) == 1
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
@pytest.mark.parametrize("hilbert,norm", [("noda", "noda"), ("circular", "noda"), ("r_compat", "paper")])
def test_fft_transform_modes_and_matmul_flag(gpu, prec, hilbert, norm):
    """Each asynchronous kernel through the FFT transform against the oracle;
    the same plan forced onto the table product agrees with both."""
    m, n = 256, 200
    S = _rand(m, n, 77)
    phi_o, psi_o = oracle.corr2d(S, hilbert=hilbert, norm=norm)
    a = _homo(S, gpu, prec=prec, hilbert=hilbert, norm=norm, basis="fourier")
    b = _homo(S, gpu, prec=prec, hilbert=hilbert, norm=norm, basis="fourier", flags=B.FLAG_TRANSFORM_MATMUL)
    assert _transform(a[2]) == 1 and _transform(b[2]) == 0
    for phi, psi, _ in (a, b):
        check_homo_structure(phi, psi)
        assert rel_fro(phi, phi_o) <= TOL[prec]
        assert rel_fro(psi, psi_o) <= TOL[prec]
    assert rel_fro(a[0], b[0]) <= TOL[prec] and rel_fro(a[1], b[1]) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16"])
@pytest.mark.parametrize("m,n", [(128, 150), (512, 70)])
def test_fft_transform_time_basis(gpu, prec, m, n):
    """Time basis with Noda's kernel: B = N Yc as an FFT correlation."""
    S = _rand(m, n, 620 + m)
    phi_o, psi_o = oracle.corr2d(S)
    a = _homo(S, gpu, prec=prec, basis="time")
    b = _homo(S, gpu, prec=prec, basis="time", flags=B.FLAG_TRANSFORM_MATMUL)
    assert _transform(a[2]) == 1 and _transform(b[2]) == 0
    for phi, psi, _ in (a, b):
        check_homo_structure(phi, psi)
        assert rel_fro(phi, phi_o) <= TOL[prec]
        assert rel_fro(psi, psi_o) <= TOL[prec]
    # A is the centred spectrum on both paths (centred by different kernels)
    assert rel_fro(a[0], b[0]) <= 1e-6 if prec != "bf16" else TOL[prec]


def test_fft_transform_hetero_ref_scaled(gpu):
    """Heterocorrelation (the left set needs no B operand), a user reference
    on one side and Pareto scaling through the FFT transform."""
    m, n1, n2 = 128, 150, 90
    S1, S2 = _rand(m, n1, 600), _rand(m, n2, 601) * 5.0
    r1 = S1[7] - 0.2
    phi_o, psi_o = oracle.corr2d(S1, S2, ref1=r1, alpha=0.5)
    phi, psi, plan, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), ref1=_t(r1, gpu), prec="split_bf16",
                                 alpha=0.5)
    assert _transform(plan) == 1
    assert rel_fro(_np(phi), phi_o) <= TOL["split_bf16"]
    assert rel_fro(_np(psi), psi_o) <= TOL["split_bf16"]


@pytest.mark.parametrize("prec", ["f64", "split_bf16"])
def test_fft_transform_f32_input_stride_and_constant_column(gpu, prec):
    """The fused centring reads FP32 input through a row stride larger than
    n, and a constant column (zero variance) stays zero under scaling -- to
    rounding: two spectral points share one complex FFT, and separating their
    spectra leaves cross-talk at the transform's rounding level."""
    import torch
    m, n, ld = 256, 150, 170
    S = _rand(m, n, 640)
    S[:, 7] = 2.5
    S32 = S.astype(np.float32)
    big = np.zeros((m, ld), dtype=np.float32)
    big[:, :n] = S32
    y = torch.as_tensor(big, device=gpu)[:, :n]
    for alpha in (0.0, 1.0):
        phi_o, psi_o = oracle.corr2d(S32.astype(np.float64), alpha=alpha)
        phi, psi, plan, _ = B.homo(y, prec=prec, alpha=alpha)
        assert _transform(plan) == 1
        ph, ps = _np(phi), _np(psi)
        assert rel_fro(ph, phi_o) <= TOL[prec] and rel_fro(ps, psi_o) <= TOL[prec]
        eps = (1e-14 if prec == "f64" else 1e-6) * np.abs(ph).max()
        assert np.abs(ph[7]).max() <= eps and np.abs(ps[7]).max() <= eps


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
def test_fft_transform_weak_columns_next_to_strong(gpu, prec):
    """Every other spectral variable varies 1e5 times less than its FFT
    partner: the block of weak variables must reach the tolerance on its
    own, i.e. the separation of the paired spectra may not leak the strong
    column's rounding into the weak one."""
    m, n = 256, 96
    rng = np.random.default_rng(650)
    S = rng.standard_normal((m, n)) + 3.0
    # no offset on the weak variables: with one, the FP64 mean's rounding
    # (any summation order) would already move their Psi by ~1e-10
    S[:, 1::2] = 1e-5 * rng.standard_normal((m, n // 2))
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, plan = _homo(S, gpu, prec=prec)
    assert _transform(plan) == 1
    w = np.arange(1, n, 2)
    assert rel_fro(phi[np.ix_(w, w)], phi_o[np.ix_(w, w)]) <= TOL[prec]
    assert rel_fro(psi[np.ix_(w, w)], psi_o[np.ix_(w, w)]) <= TOL[prec]
    assert rel_fro(phi, phi_o) <= TOL[prec] and rel_fro(psi, psi_o) <= TOL[prec]


def test_fft_transform_after_interpolation(gpu):
    m_in, m_out, n = 90, 128, 140
    t = _uneven(m_in, 610)
    S = _rand(m_in, n, 611)
    phi_o, psi_o = oracle.corr2d(oracle.interpolate(S, t, m_out, "spline"))
    phi, psi, plan = _homo(S, gpu, prec="f32", interp="spline", t_in=t, m_out=m_out)
    assert _transform(plan) == 1
    assert rel_fro(phi, phi_o) <= TOL["f32"] and rel_fro(psi, psi_o) <= TOL["f32"]


# --------------------------------------------------------------------------
# Edge sizes: long perturbation axes (centring without the register cache,
# the largest m), and a very wide heterocorrelation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "fp8_e4m3"])
@pytest.mark.parametrize("m,n", [(300, 190), (1000, 70), (4096, 33)])
def test_long_perturbation_axis(gpu, prec, m, n):
    S = _rand(m, n, 500 + m)
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, _ = _homo(S, gpu, prec=prec)
    check_homo_structure(phi, psi)
    assert rel_fro(phi, phi_o) <= TOL[prec]
    assert rel_fro(psi, psi_o) <= TOL[prec]


def test_max_n_heterocorrelation(gpu):
    """n1 at the plan's limit (2^24 spectral points): 64-bit offsets through
    the workspace, the operand planes and the output; sampled entries,
    including the last rows, against the oracle."""
    m, n1, n2 = 3, 1 << 24, 3
    rng = np.random.default_rng(520)
    S1 = rng.standard_normal((m, n1)) + 1.0
    S2 = rng.standard_normal((m, n2)) - 2.0
    i = np.concatenate([rng.integers(0, n1, 3000), [n1 - 1, n1 - 2, 0, (1 << 23) + 5]])
    j = np.concatenate([rng.integers(0, n2, 3000), [n2 - 1, 0, 1, 2]])
    po, qo = oracle.corr2d_entries(S1, i, j, S2=S2)
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec="f32")
    import torch
    idx = torch.as_tensor(i * n2 + j, device=gpu)
    gp = phi.reshape(-1)[idx].double().cpu().numpy()
    gq = psi.reshape(-1)[idx].double().cpu().numpy()
    assert rel_fro(gp, po) <= TOL["f32"]
    assert rel_fro(gq, qo) <= TOL["f32"]


def test_fft_transform_large_n(gpu):
    """The FFT transform (m = 128) over 2^22 spectral points (262144
    workgroups, operand planes of 2^30 bytes); sampled entries, including the
    last rows, against the oracle."""
    m, n1, n2 = 128, 1 << 22, 5
    rng = np.random.default_rng(530)
    S1 = rng.standard_normal((m, n1)).astype(np.float32).astype(np.float64) + 1.0
    S2 = rng.standard_normal((m, n2)) - 2.0
    i = np.concatenate([rng.integers(0, n1, 2000), [n1 - 1, n1 - 2, n1 - 3, 0]])
    j = np.concatenate([rng.integers(0, n2, 2000), [n2 - 1, 0, 3, 1]])
    po, qo = oracle.corr2d_entries(S1, i, j, S2=S2)
    phi, psi, plan, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec="split_bf16")
    assert _transform(plan) == 1
    import torch
    idx = torch.as_tensor(i * n2 + j, device=gpu)
    gp = phi.reshape(-1)[idx].double().cpu().numpy()
    gq = psi.reshape(-1)[idx].double().cpu().numpy()
    assert rel_fro(gp, po) <= TOL["split_bf16"]
    assert rel_fro(gq, qo) <= TOL["split_bf16"]


def test_wide_heterocorrelation(gpu):
    m, n1, n2 = 6, 120000, 37
    S1, S2 = _rand(m, n1, 510), _rand(m, n2, 511)
    rng = np.random.default_rng(512)
    i, j = rng.integers(0, n1, 4000), rng.integers(0, n2, 4000)
    i[:3] = [n1 - 1, 0, n1 - 1]
    j[:3] = [n2 - 1, n2 - 1, 0]
    po, qo = oracle.corr2d_entries(S1, i, j, S2=S2)
    phi, psi, _, _ = B.hetero(_t(S1, gpu), _t(S2, gpu), prec="f32")
    gp, gq = _np(phi), _np(psi)
    assert rel_fro(gp[i, j], po) <= TOL["f32"]
    assert rel_fro(gq[i, j], qo) <= TOL["f32"]
