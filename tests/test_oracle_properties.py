"""Property tests of the FP64 oracle over random shapes (hypothesis), and a
brute-force cross-check against pure-Python math.fsum sums on tiny inputs.

The pins in test_oracle_pins.py tie each oracle function to what the paper
and the mathematics fix; these tests sweep the shapes and references the
pins do not enumerate (m in [2, 40], n in [1, 64], heterocorrelation with
n1 != n2), so that an index or stride mistake that only shows for some
shapes fails here.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True)


def _spectra(m, n, seed, offset=0.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * rng.uniform(0.1, 10.0) + offset


def _scale(a):
    return max(1.0, float(np.abs(a).max()))


# --------------------------------------------------------------------------
# Brute force: Noda's formulas (Sec. 2 Eqs. (disHTsyn), (disHTasyn)) written
# as plain loops with correctly rounded sums
# --------------------------------------------------------------------------
def _brute(S1, S2=None, ref1=None, ref2=None):
    S2_ = S1 if S2 is None else S2
    m = len(S1)

    def centred(S, ref):
        n = len(S[0])
        mean = [ref[j] if ref is not None else math.fsum(S[k][j] for k in range(m)) / m for j in range(n)]
        return [[S[k][j] - mean[j] for j in range(n)] for k in range(m)]

    Y1 = centred(S1, ref1)
    Y2 = Y1 if S2 is None else centred(S2_, ref2)
    n1, n2 = len(Y1[0]), len(Y2[0])
    # (N y)_k = sum_{l != k} y_l / (pi (l - k))
    NY2 = [[math.fsum(Y2[l][j] / (math.pi * (l - k)) for l in range(m) if l != k) for j in range(n2)]
           for k in range(m)]
    phi = [[math.fsum(Y1[k][i] * Y2[k][j] for k in range(m)) / (m - 1) for j in range(n2)] for i in range(n1)]
    psi = [[math.fsum(Y1[k][i] * NY2[k][j] for k in range(m)) / (m - 1) for j in range(n2)] for i in range(n1)]
    return np.array(phi), np.array(psi)


small = st.integers(min_value=2, max_value=6)
smalln = st.integers(min_value=1, max_value=6)
vals = st.floats(min_value=-10.0, max_value=10.0, allow_nan=False, allow_infinity=False)


@SETTINGS
@given(m=small, n1=smalln, n2=smalln, data=st.data(), hetero=st.booleans(), use_ref=st.booleans())
def test_brute_force_fsum(m, n1, n2, data, hetero, use_ref):
    S1 = [[data.draw(vals) for _ in range(n1)] for _ in range(m)]
    S2 = [[data.draw(vals) for _ in range(n2)] for _ in range(m)] if hetero else None
    r1 = [data.draw(vals) for _ in range(n1)] if use_ref else None
    r2 = [data.draw(vals) for _ in range(n2)] if (use_ref and hetero) else None
    bp, bq = _brute(S1, S2, r1, r2)
    op, oq = oracle.corr2d(np.array(S1), None if S2 is None else np.array(S2),
                           ref1=None if r1 is None else np.array(r1),
                           ref2=None if r2 is None else np.array(r2))
    tol = 1e-12 * max(1.0, float(np.abs(bp).max()), float(np.abs(bq).max()))
    assert np.abs(op - bp).max() <= tol
    assert np.abs(oq - bq).max() <= tol


# --------------------------------------------------------------------------
# Invariants over random shapes
# --------------------------------------------------------------------------
ms = st.integers(min_value=2, max_value=40)
ns = st.integers(min_value=1, max_value=64)
seeds = st.integers(min_value=0, max_value=2 ** 31 - 1)


@SETTINGS
@given(m=ms, n=ns, seed=seeds, use_ref=st.booleans())
def test_structure_and_autopower(m, n, seed, use_ref):
    """Phi symmetric, Psi antisymmetric with a zero diagonal, and the Phi
    diagonal the autopower sum (y - ref)^2 / (m - 1) (Eq. (stdev) squared
    for the mean reference)."""
    S = _spectra(m, n, seed)
    ref = S[seed % m] + 0.5 if use_ref else None
    phi, psi = oracle.corr2d(S, ref1=ref)
    assert np.array_equal(phi, phi.T)
    sc = _scale(psi)
    assert np.abs(psi + psi.T).max() <= 1e-12 * sc
    assert np.all(np.diag(psi) == 0.0) or np.abs(np.diag(psi)).max() <= 1e-12 * sc
    r = S.mean(axis=0) if ref is None else ref
    auto = np.array([math.fsum((S[:, j] - r[j]) ** 2) for j in range(n)]) / (m - 1)
    assert np.abs(np.diag(phi) - auto).max() <= 1e-12 * _scale(auto)


@SETTINGS
@given(m=ms, n=ns, seed=seeds)
def test_offset_and_scale(m, n, seed):
    """A constant added to each spectral variable disappears with the mean;
    the result is bilinear in the spectra."""
    S = _spectra(m, n, seed)
    off = np.random.default_rng(seed + 1).uniform(-50, 50, n)
    p0, q0 = oracle.corr2d(S)
    p1, q1 = oracle.corr2d(S + off)
    assert np.abs(p1 - p0).max() <= 1e-9 * _scale(p0)
    assert np.abs(q1 - q0).max() <= 1e-9 * _scale(p0)
    p2, q2 = oracle.corr2d(-3.0 * S)
    assert np.abs(p2 - 9.0 * p0).max() <= 1e-12 * _scale(9.0 * p0)
    assert np.abs(q2 - 9.0 * q0).max() <= 1e-12 * _scale(9.0 * p0)


@SETTINGS
@given(m=ms, n1=ns, n2=ns, seed=seeds)
def test_hetero_blocks_and_time_reversal(m, n1, n2, seed):
    """The heterocorrelation of [S1 | S2] with itself holds the cross blocks;
    reversing the perturbation order negates Psi and keeps Phi."""
    S1, S2 = _spectra(m, n1, seed), _spectra(m, n2, seed + 7)
    ph, qh = oracle.corr2d(S1, S2)
    pa, qa = oracle.corr2d(np.hstack([S1, S2]))
    sc = _scale(pa)
    assert np.abs(ph - pa[:n1, n1:]).max() <= 1e-12 * sc
    assert np.abs(qh - qa[:n1, n1:]).max() <= 1e-12 * sc
    pr, qr = oracle.corr2d(S1[::-1], S2[::-1])
    assert np.abs(pr - ph).max() <= 1e-12 * sc
    assert np.abs(qr + qh).max() <= 1e-12 * sc


@SETTINGS
@given(m=ms, n1=ns, n2=ns, seed=seeds, extra=st.integers(min_value=0, max_value=9))
def test_fourier_routes_against_direct(m, n1, n2, seed, extra):
    """Parseval: the m-point Fourier route's Phi equals the direct Phi; the
    zero-padded route of any length L >= 2m - 1 gives Phi and Psi."""
    Y1, _ = oracle.dynamic(_spectra(m, n1, seed))
    Y2, _ = oracle.dynamic(_spectra(m, n2, seed + 3))
    pd, qd = oracle.corr_ht(Y1, Y2)
    pc, _ = oracle.corr_ft_circular(Y1, Y2, oracle.norm_factor(m))
    sc = _scale(pd)
    assert np.abs(pc - pd).max() <= 1e-11 * sc
    pp, qp = oracle.corr_ft_padded(Y1, Y2, L=2 * m - 1 + extra)
    assert np.abs(pp - pd).max() <= 1e-11 * sc
    assert np.abs(qp - qd).max() <= 1e-11 * sc


@SETTINGS
@given(m=ms, n=ns, seed=seeds)
def test_paper_norm_ratio(m, n, seed):
    """PAPER over NODA normalization is m / pi (Eq. (disint2d) against Eqs.
    (disHTsyn), (disHTasyn))."""
    S = _spectra(m, n, seed)
    p0, q0 = oracle.corr2d(S)
    p1, q1 = oracle.corr2d(S, norm="paper")
    assert np.abs(p1 - p0 * m / math.pi).max() <= 1e-12 * _scale(p1)
    assert np.abs(q1 - q0 * m / math.pi).max() <= 1e-12 * _scale(p1)


def test_property_suite_is_deterministic():
    """derandomize=True: the examples are the same on every run."""
    assert SETTINGS.derandomize


if __name__ == "__main__":  # pragma: no cover
    pytest.main([__file__])
