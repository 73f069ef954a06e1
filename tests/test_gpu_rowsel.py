"""Row-selective split (CORR2D_FLAG_SPLIT_ROWS) against the oracle and
against the full split and the plain formats it reduces to.

The low plane enters only the products of the packed Fourier rows (pairs of
16-row K blocks) that hold most of the operands' energy; the others are
multiplied in the high plane alone.  Each call chooses the rows from the
target error it is given (Sec. 4.2: the Hermitian half spectrum of a band
spectrum's dynamic spectra is concentrated in the low frequencies)."""
import numpy as np
import pytest

import oracle
from paper_1808_00685_amd import binding as B
from paper_1808_00685_amd import synth

from .gpu_helpers import TOL, check_homo_structure, rel_fro

pytestmark = pytest.mark.gpu
SPLITS = ["split_bf16", "split_f16"]


def _t(a, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _check_selection(sel, kp):
    nsel, order = sel
    nkb = kp // 16
    assert 0 <= nsel <= nkb and nsel % 2 == 0
    assert sorted(order) == list(range(nkb))
    # pairs of K blocks stay together, in their natural order
    assert all(order[2 * r] % 2 == 0 and order[2 * r + 1] == order[2 * r] + 1 for r in range(nkb // 2))
    return nsel


@pytest.mark.parametrize("prec", SPLITS)
@pytest.mark.parametrize("m,n", [(256, 1500), (181, 700), (64, 300)])
def test_tiny_target_is_the_full_split(gpu, prec, m, n):
    """A target no row can be dropped for selects every row pair and keeps
    the natural order: the same bits as the full split."""
    S, _ = synth.bands(m, n, 16, seed=synth.BASE_SEED + 3100 + m)
    y = _t(S, gpu)
    phi, psi, plan, ws = B.homo(y, prec=prec, flags=B.FLAG_SPLIT_ROWS, split_tol=1e-30)
    nsel = _check_selection(B.selection(ws, plan), plan.info.k_pad)
    assert nsel == plan.info.k_pad // 16
    assert B.selection(ws, plan)[1] == list(range(plan.info.k_pad // 16))
    fphi, fpsi, _, _ = B.homo(y, prec=prec, basis="fourier")
    assert np.array_equal(_np(phi), _np(fphi)) and np.array_equal(_np(psi), _np(fpsi))


@pytest.mark.parametrize("prec,plain", [("split_bf16", "bf16"), ("split_f16", "f16")])
@pytest.mark.parametrize("m,n", [(256, 1500), (96, 700)])
def test_loose_target_is_the_high_plane_alone(gpu, prec, plain, m, n):
    """A target every row can be dropped for selects none and keeps the
    natural order: the same bits as the plain format in the Fourier basis
    (the high plane is that format's rounding, with the same scales)."""
    S, _ = synth.bands(m, n, 16, seed=synth.BASE_SEED + 3200 + m)
    y = _t(S, gpu)
    phi, psi, plan, ws = B.homo(y, prec=prec, flags=B.FLAG_SPLIT_ROWS, split_tol=1e6, tile=3)
    nsel, order = B.selection(ws, plan)
    assert nsel == 0 and order == list(range(plan.info.k_pad // 16))
    pphi, ppsi, _, _ = B.homo(y, prec=plain, basis="fourier", tile=3)
    assert np.array_equal(_np(phi), _np(pphi)) and np.array_equal(_np(psi), _np(ppsi))


@pytest.mark.parametrize("prec", SPLITS)
@pytest.mark.parametrize("m,n,flags", [(256, 3000, 0), (256, 3000, B.FLAG_TRANSFORM_MATMUL),
                                       (128, 2500, 0), (200, 2000, 0), (96, 1111, 0)])
def test_row_select_parity_band_spectra(gpu, prec, m, n, flags):
    """Band spectra (the benchmark's generator) through both transforms: the
    stated target 1e-5 holds against the oracle on the full matrices, the
    record is a valid selection, and fewer than all pairs are selected."""
    S, _ = synth.bands(m, n, 48, seed=synth.BASE_SEED + 3300 + m, log_amplitude=True,
                       relative_b=True, sigma=1e-4, a_range=(1e-3, 1e2), b_range=(0.05, 0.5),
                       drift=(-0.3, 0.3))
    phi_o, psi_o = oracle.corr2d(S)
    phi, psi, plan, ws = B.homo(_t(S, gpu), prec=prec, flags=flags | B.FLAG_SPLIT_ROWS)
    assert plan.info.transform == (0 if flags or m & (m - 1) else 1)
    phi, psi = _np(phi), _np(psi)
    check_homo_structure(phi, psi)
    nsel = _check_selection(B.selection(ws, plan), plan.info.k_pad)
    e_phi, e_psi = rel_fro(phi, phi_o), rel_fro(psi, psi_o)
    print(f"rowsel {prec} m={m} n={n} flags={flags}: {nsel}/{plan.info.k_pad // 16} K blocks split, "
          f"phi {e_phi:.2e} psi {e_psi:.2e}")
    assert e_phi <= 1e-5 and e_psi <= 1e-5
    if prec == "split_f16":
        assert nsel < plan.info.k_pad // 16


@pytest.mark.parametrize("prec", SPLITS)
def test_row_select_heterocorrelation(gpu, prec):
    """The heterocorrelation workload's generator at a reduced size: rows
    ranked by the left A and both right operands."""
    S1, S2, _ = synth.workload_hetero(n1=2048, n2=512)
    phi_o, psi_o = oracle.corr2d(S1, S2)
    phi, psi, plan, ws = B.hetero(_t(S1, gpu), _t(S2, gpu), prec=prec, flags=B.FLAG_SPLIT_ROWS)
    nsel = _check_selection(B.selection(ws, plan), plan.info.k_pad)
    e_phi, e_psi = rel_fro(_np(phi), phi_o), rel_fro(_np(psi), psi_o)
    print(f"rowsel hetero {prec}: {nsel}/{plan.info.k_pad // 16} K blocks split, phi {e_phi:.2e} psi {e_psi:.2e}")
    assert e_phi <= 1e-5 and e_psi <= 1e-5


@pytest.mark.parametrize("prec", SPLITS)
def test_row_select_target_orders_the_selection(gpu, prec):
    """Tighter targets select at least as many row pairs (the chosen pairs
    are a prefix of one ranking), and the error follows."""
    S, _ = synth.bands(256, 2000, 32, seed=synth.BASE_SEED + 3400, log_amplitude=True,
                       relative_b=True, sigma=1e-4, a_range=(1e-3, 1e2))
    phi_o, _ = oracle.corr2d(S)
    y = _t(S, gpu)
    floor = {"split_bf16": 1e-5, "split_f16": 1e-6}[prec]   # the full split's own error, about
    prev_n, prev_order = -1, None
    for tol in (1e-2, 1e-4, 1e-5, 1e-7):
        phi, psi, plan, ws = B.homo(y, prec=prec, flags=B.FLAG_SPLIT_ROWS, split_tol=tol)
        nsel, order = B.selection(ws, plan)
        assert nsel >= prev_n
        if prev_order is not None and 0 < prev_n and nsel < len(order):
            assert order[:prev_n] == prev_order[:prev_n]
        prev_n, prev_order = nsel, order
        assert rel_fro(_np(phi), phi_o) <= max(tol, floor)
