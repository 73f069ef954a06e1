"""The allocation-free homocorrelation entry point (corr2d_homo_noalloc,
the library's fixed device scratch as the workspace) against corr2d_homo
with a caller workspace: two calls in a row, the second on a smaller input,
so the second runs on scratch that still holds the first call's data."""
import numpy as np
import pytest

from paper_1808_00685_amd import binding as B
from paper_1808_00685_amd import synth

pytestmark = pytest.mark.gpu


def _pair(gpu, S, prec, layout):
    import torch
    m, n = S.shape
    y = torch.as_tensor(S, device=gpu)
    out_dtype = "f64" if prec == "f64" else "f32"
    plan = B.Plan(m=m, n1=n, n2=0, prec=prec, out_layout=layout, in_dtype="f64", out_dtype=out_dtype)
    assert plan.ws_bytes <= B.NOALLOC_SCRATCH_BYTES
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    numel = B.out_elements(layout, n)
    outs = []
    for use_scratch in (True, False):
        phi = torch.full((numel,), float("nan"), dtype=tdt, device=gpu)
        psi = torch.full((numel,), float("nan"), dtype=tdt, device=gpu)
        if use_scratch:
            B.corr2d_homo_noalloc(plan.handle, y, None, phi, psi)
        else:
            ws = plan.workspace(gpu)
            B.corr2d_homo(plan.handle, y, None, phi, psi, ws)
        torch.cuda.synchronize()
        outs.append((phi, psi))
    return outs


def _same(a, b):
    """Bit-for-bit equal, the padding slots of an upper layout (left NaN by
    both calls, never written) included."""
    import torch
    both_nan = torch.isnan(a) & torch.isnan(b)
    return bool(torch.all((a == b) | both_nan))


def test_noalloc_matches_workspace_entry_on_two_calls(gpu):
    import torch
    # first call: the m=256, n=16384 workload (radix FFT transform, split-BF16)
    S, _ = synth.workload_large()
    (a_phi, a_psi), (b_phi, b_psi) = _pair(gpu, S, "split_bf16", "upper_aligned")
    n = S.shape[1]
    assert int(torch.isnan(a_phi).sum()) == a_phi.numel() - n * (n + 1) // 2
    assert _same(a_phi, b_phi) and _same(a_psi, b_psi)
    del a_phi, a_psi, b_phi, b_psi
    # second call, smaller: odd m (table-product transform), FP32, full layout
    S2, _ = synth.bands(37, 3000, 12, seed=synth.BASE_SEED + 777)
    (a_phi, a_psi), (b_phi, b_psi) = _pair(gpu, S2, "f32", "full")
    assert not torch.isnan(a_phi).any() and not torch.isnan(a_psi).any()
    assert torch.equal(a_phi, b_phi) and torch.equal(a_psi, b_psi)
