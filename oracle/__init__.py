"""FP64 CPU oracle for generalized two-dimensional correlation analysis.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the HIP product path (``paper_1808_00685_amd``)
and never imports it; the product path never imports this package.

The numerical work lives in ``oracle.c`` (plain C, double precision, natural
summation order, OpenMP over independent output rows).  This module only
marshals numpy arrays and combines the paper's normalization readings:

* ``hilbert="noda"``: Noda's direct formulas, Sec. 2 Eqs. (disHTsyn), (disHT),
  (HilbNoda), (disHTasyn) -- synchronous  Y1^T Y2 / (m-1), asynchronous
  Y1^T N Y2 / (m-1) with the Hilbert-Noda matrix N.
* ``hilbert="circular"``: the m-point Fourier route, Sec. 2 Eqs. (disFT),
  (disint2d), (symmeFT) with the Hermitian-complete half spectrum of Sec. 4.2.
* Normalization ``norm`` is the factor cF applied to the Hermitian-weighted
  Fourier sum (Sec. 4.2, the ``Norm`` argument): "noda" cF = 1/(m(m-1)), which
  makes the synchronous spectrum equal Y^T Y/(m-1); "paper" cF = 1/(pi(m-1)),
  the paper's default ``Norm``; "custom" cF = ``norm_value``.  Since the
  weighted Fourier sum of real data is m times the time-domain sum (Parseval),
  the direct route under norm cF is the "noda" result times cF*m*(m-1).
* ``hilbert="r_compat"``: the Fourier route exactly as the R code of Sec. 4.2
  evaluates it -- the bin list (1..m-1) %/% 2 with its repeats (DC once,
  the top bin once for odd m, the Nyquist bin of even m left out).
* ``interpolate`` (Sec. 4.1): spectra resampled on N equidistant perturbation
  values, piecewise linear or with the FMM cubic spline (the default method of
  R's splinefun, which the paper names as the default interpolation).
* Scaling ``alpha`` (Sec. 2 Eqs. (stdev), (scalesyn), (scaleasyn)): the result
  divided by (sigma_1 sigma_2)^alpha, sigma per spectral variable from the
  dynamic spectra in use; a variable with sigma = 0 is left unscaled.

Parity pins (tests/test_oracle_pins.py) tie every function here to closed
forms, invariants and an independent padded-Fourier algorithm.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

GCC_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB_PATH, _SRC, "-lm"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (plain gcc, no HIP)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        subprocess.run(GCC_CMD, check=True)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        cl = ctypes.c_long
        L.oracle_dynamic.argtypes = [cl, cl, dp, cl, dp, dp, dp]
        L.oracle_hilbert_noda.argtypes = [cl, dp]
        L.oracle_noda_transform.argtypes = [cl, cl, dp, dp]
        L.oracle_corr_ht.argtypes = [cl, cl, cl, dp, dp, dp, dp]
        L.oracle_corr_ht_entries.argtypes = [cl, cl, cl, dp, dp, cl, lp, lp, dp, dp]
        L.oracle_dft.argtypes = [cl, cl, dp, dp, dp]
        L.oracle_corr_ft_circular.argtypes = [cl, cl, cl, dp, dp, ctypes.c_double, dp, dp]
        L.oracle_corr_ft_padded.argtypes = [cl, cl, cl, dp, dp, cl, dp, dp]
        L.oracle_corr_ft_circular_entries.argtypes = [cl, cl, cl, dp, dp, ctypes.c_double,
                                                      cl, lp, lp, dp, dp]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def set_threads(t: int) -> None:
    """Threads for the oracle's later parallel loops (timing only)."""
    lib().oracle_set_threads(int(t))


# --------------------------------------------------------------------------
# Building blocks (each follows one equation of the paper)
# --------------------------------------------------------------------------
def dynamic(S, ref=None):
    """Dynamic spectra, Sec. 2 Eqs. (dynspec), (ref); Sec. 4.2.

    S: (m, n) spectra, perturbation steps by rows.  ref: optional (n,)
    reference spectrum; default the perturbation mean.  Returns (Y, r).
    """
    S = _f64(S)
    m, n = S.shape
    Y = np.empty((m, n))
    r = np.empty(n)
    rp = None
    if ref is not None:
        ref = _f64(ref)
        assert ref.shape == (n,)
        rp = _p(ref)
    lib().oracle_dynamic(m, n, _p(S), n, rp, _p(Y), _p(r))
    return Y, r


def hilbert_noda(m):
    """Hilbert-Noda matrix, Sec. 2 Eq. (HilbNoda)."""
    N = np.empty((m, m))
    lib().oracle_hilbert_noda(m, _p(N))
    return N


def noda_transform(Y):
    """z = N y for every column, Sec. 2 Eq. (disHT)."""
    Y = _f64(Y)
    m, n = Y.shape
    Z = np.empty((m, n))
    lib().oracle_noda_transform(m, n, _p(Y), _p(Z))
    return Z


def corr_ht(Y1, Y2):
    """Direct route on dynamic spectra; returns full (phi, psi)."""
    Y1, Y2 = _f64(Y1), _f64(Y2)
    m, n1 = Y1.shape
    m2, n2 = Y2.shape
    assert m == m2 and m >= 2
    phi = np.empty((n1, n2))
    psi = np.empty((n1, n2))
    lib().oracle_corr_ht(m, n1, n2, _p(Y1), _p(Y2), _p(phi), _p(psi))
    return phi, psi


def corr_ht_block(Y1, Y2, r0, r1, c0, c1):
    """Rows r0..r1-1 and columns c0..c1-1 of corr_ht(Y1, Y2): the direct
    route on those columns of the dynamic spectra (N acts on each column of
    the second set by itself, Eq. (disHT)), for outputs too large to hold."""
    Y1, Y2 = _f64(Y1), _f64(Y2)
    return corr_ht(Y1[:, r0:r1], Y2[:, c0:c1])


def corr_ht_entries(Y1, Y2, rows, cols):
    """Selected entries (rows[t], cols[t]) of the direct route."""
    Y1, Y2 = _f64(Y1), _f64(Y2)
    m, n1 = Y1.shape
    _, n2 = Y2.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    assert rows.shape == cols.shape
    assert (rows >= 0).all() and (rows < n1).all() and (cols >= 0).all() and (cols < n2).all()
    phi = np.empty(rows.shape[0])
    psi = np.empty(rows.shape[0])
    lib().oracle_corr_ht_entries(m, n1, n2, _p(Y1), _p(Y2), rows.shape[0], _lp(rows), _lp(cols),
                                 _p(phi), _p(psi))
    return phi, psi


def dft(Y):
    """m-point DFT along the perturbation axis, Sec. 2 Eq. (disFT)."""
    Y = _f64(Y)
    m, n = Y.shape
    re = np.empty((m, n))
    im = np.empty((m, n))
    lib().oracle_dft(m, n, _p(Y), _p(re), _p(im))
    return re + 1j * im


def corr_ft_circular(Y1, Y2, cF):
    """m-point Fourier route with Hermitian-complete half spectrum."""
    Y1, Y2 = _f64(Y1), _f64(Y2)
    m, n1 = Y1.shape
    _, n2 = Y2.shape
    phi = np.empty((n1, n2))
    psi = np.empty((n1, n2))
    lib().oracle_corr_ft_circular(m, n1, n2, _p(Y1), _p(Y2), float(cF), _p(phi), _p(psi))
    return phi, psi


def r_bins(m):
    """Bins the R code of Sec. 4.2 keeps from each m-point FFT: with R's
    precedence ``1:(m-1) %/% 2 + 1`` is (1..m-1) integer-divided by 2, plus 1
    (1-based), i.e. 0-based bins floor(j/2) for j = 1..m-1, repeats kept."""
    return np.array([j // 2 for j in range(1, m)], dtype=np.int64)


def corr_ft_r(Y1, Y2, cF):
    """The R package's Fourier route as printed (Sec. 4.2): cF times the sum,
    over the bin list r_bins(m) with its repeats, of F1(bin) conj(F2(bin)),
    F the m-point DFT of each dynamic spectrum; real part Phi, imaginary Psi."""
    m = np.asarray(Y1).shape[0]
    F1 = dft(Y1)
    F2 = F1 if Y2 is Y1 else dft(Y2)
    C = np.zeros((F1.shape[1], F2.shape[1]), dtype=np.complex128)
    for b in r_bins(m):
        C += np.outer(F1[b], np.conj(F2[b]))
    C *= cF
    return C.real.copy(), C.imag.copy()


def corr_ft_circular_entries(Y1, Y2, cF, rows, cols):
    Y1, Y2 = _f64(Y1), _f64(Y2)
    m, n1 = Y1.shape
    _, n2 = Y2.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    assert (rows >= 0).all() and (rows < n1).all() and (cols >= 0).all() and (cols < n2).all()
    phi = np.empty(rows.shape[0])
    psi = np.empty(rows.shape[0])
    lib().oracle_corr_ft_circular_entries(m, n1, n2, _p(Y1), _p(Y2), float(cF), rows.shape[0],
                                          _lp(rows), _lp(cols), _p(phi), _p(psi))
    return phi, psi


def corr_ft_padded(Y1, Y2, L=None):
    """Zero-padded L-point Fourier route (L >= 2m-1) reproducing the direct route."""
    Y1, Y2 = _f64(Y1), _f64(Y2)
    m, n1 = Y1.shape
    _, n2 = Y2.shape
    if L is None:
        L = 2 * m
    phi = np.empty((n1, n2))
    psi = np.empty((n1, n2))
    lib().oracle_corr_ft_padded(m, n1, n2, _p(Y1), _p(Y2), int(L), _p(phi), _p(psi))
    return phi, psi


# --------------------------------------------------------------------------
# Whole calculation (the paper's corr2d(): reference, dynamic spectra, route)
# --------------------------------------------------------------------------
def norm_factor(m, norm="noda", norm_value=None):
    """cF, the factor applied to the Hermitian-weighted Fourier sum."""
    if norm == "noda":
        return 1.0 / (m * (m - 1))
    if norm == "paper":
        return 1.0 / (math.pi * (m - 1))
    if norm == "custom":
        return float(norm_value)
    raise ValueError(norm)


def fmm_spline_second_derivatives(x, y):
    """Second derivatives M at the knots of the cubic spline through (x, y)
    with Forsythe-Malcolm-Moler end conditions: the spline's third derivative
    on the first (last) interval equals that of the cubic through the first
    (last) four points, 6 times their third divided difference.  Two points
    give the straight line (M = 0), three the parabola through them.  Solved
    as a dense linear system in FP64 (the plain definition)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    if n < 3:
        return np.zeros(n)
    h = np.diff(x)
    d = np.diff(y) / h
    A = np.zeros((n, n))
    r = np.zeros(n)
    for i in range(1, n - 1):
        A[i, i - 1] = h[i - 1]
        A[i, i] = 2.0 * (h[i - 1] + h[i])
        A[i, i + 1] = h[i]
        r[i] = 6.0 * (d[i] - d[i - 1])
    if n == 3:
        third_l = third_r = 0.0
    else:
        def dd3(xs, ys):
            d1 = np.diff(ys) / np.diff(xs)
            d2 = np.diff(d1) / (xs[2:] - xs[:-2])
            return (d2[1] - d2[0]) / (xs[3] - xs[0])
        third_l = 6.0 * dd3(x[:4], y[:4])
        third_r = 6.0 * dd3(x[-4:], y[-4:])
    # (M1 - M0)/h0 = third_l, (M[n-1] - M[n-2])/h[n-2] = third_r
    A[0, 0], A[0, 1], r[0] = -1.0, 1.0, third_l * h[0]
    A[n - 1, n - 2], A[n - 1, n - 1], r[n - 1] = -1.0, 1.0, third_r * h[-1]
    return np.linalg.solve(A, r)


def fmm_spline_eval(x, y, M, t):
    """Value at t of the cubic spline with knots x, values y and second
    derivatives M (t inside [x0, x_last])."""
    x = np.asarray(x, dtype=np.float64)
    i = np.clip(np.searchsorted(x, t, side="right") - 1, 0, len(x) - 2)
    h = x[i + 1] - x[i]
    a, b = x[i + 1] - t, t - x[i]
    return (M[i] * a ** 3 / (6 * h) + M[i + 1] * b ** 3 / (6 * h) +
            (y[i] / h - M[i] * h / 6) * a + (y[i + 1] / h - M[i + 1] * h / 6) * b)


def interpolate(S, t_in, N, method="spline"):
    """Spectra on N equidistant perturbation values over [min t, max t]
    (Sec. 4.1: seq(min(Time), max(Time), length.out = N), then each spectral
    variable interpolated along t): method "linear" (piecewise linear) or
    "spline" (the FMM cubic spline).  t_in strictly increasing."""
    S = np.asarray(S, dtype=np.float64)
    t_in = np.asarray(t_in, dtype=np.float64)
    T = np.linspace(t_in[0], t_in[-1], int(N))
    out = np.empty((len(T), S.shape[1]))
    for c in range(S.shape[1]):
        if method == "linear":
            out[:, c] = np.interp(T, t_in, S[:, c])
        elif method == "spline":
            M = fmm_spline_second_derivatives(t_in, S[:, c])
            out[:, c] = fmm_spline_eval(t_in, S[:, c], M, T)
        else:
            raise ValueError(method)
    return out


def band_sd(Y):
    """sigma_nu of every spectral variable (column) of the dynamic spectra Y,
    Sec. 2 Eq. (stdev): sqrt(sum_j Y[j, nu]^2 / (m - 1)), Y already centred on
    the reference in use."""
    Y = np.asarray(Y, dtype=np.float64)
    return np.sqrt(np.sum(Y * Y, axis=0) / (Y.shape[0] - 1))


def scaling_factors(sd, alpha):
    """sigma^-alpha per spectral variable; 1 where sigma = 0 (that variable's
    dynamic spectrum is zero, so leaving it unscaled changes nothing)."""
    sd = np.asarray(sd, dtype=np.float64)
    f = np.ones_like(sd)
    nz = sd > 0
    f[nz] = sd[nz] ** (-float(alpha))
    return f


def corr2d(S1, S2=None, ref1=None, ref2=None, hilbert="noda", norm="noda", norm_value=None,
           alpha=0.0):
    """Full (phi, psi) for homocorrelation (S2 None) or heterocorrelation.

    alpha != 0 applies the scaling of Sec. 2 Eqs. (scalesyn), (scaleasyn), read
    as phi / (sigma_1 sigma_2)^alpha (Pearson alpha = 1, Pareto 0.5) with the
    sigma of Eq. (stdev) per spectral variable of each set."""
    Y1, _ = dynamic(S1, ref1)
    Y2 = Y1 if S2 is None else dynamic(S2, ref2)[0]
    m = Y1.shape[0]
    cF = norm_factor(m, norm, norm_value)
    if hilbert == "noda":
        phi, psi = corr_ht(Y1, Y2)
        f = cF * m * (m - 1)
        if f != 1.0:
            phi = phi * f
            psi = psi * f
    elif hilbert == "circular":
        phi, psi = corr_ft_circular(Y1, Y2, cF)
    elif hilbert == "r_compat":
        phi, psi = corr_ft_r(Y1, Y2 if S2 is not None else Y1, cF)
    else:
        raise ValueError(hilbert)
    if alpha != 0.0:
        w = np.outer(scaling_factors(band_sd(Y1), alpha), scaling_factors(band_sd(Y2), alpha))
        phi = phi * w
        psi = psi * w
    return phi, psi


def corr2d_entries(S1, rows, cols, S2=None, ref1=None, ref2=None, hilbert="noda",
                   norm="noda", norm_value=None, alpha=0.0):
    """Selected entries of corr2d(); the dynamic spectra are formed in full."""
    Y1, _ = dynamic(S1, ref1)
    Y2 = Y1 if S2 is None else dynamic(S2, ref2)[0]
    m = Y1.shape[0]
    cF = norm_factor(m, norm, norm_value)
    if hilbert == "noda":
        phi, psi = corr_ht_entries(Y1, Y2, rows, cols)
        f = cF * m * (m - 1)
        if f != 1.0:
            phi = phi * f
            psi = psi * f
    elif hilbert == "circular":
        phi, psi = corr_ft_circular_entries(Y1, Y2, cF, rows, cols)
    elif hilbert == "r_compat":
        rows, cols = np.asarray(rows), np.asarray(cols)
        F1 = dft(Y1)
        F2 = F1 if S2 is None else dft(Y2)
        c = np.zeros(len(rows), dtype=np.complex128)
        for b in r_bins(m):
            c += F1[b][rows] * np.conj(F2[b][cols])
        c *= cF
        phi, psi = c.real.copy(), c.imag.copy()
    else:
        raise ValueError(hilbert)
    if alpha != 0.0:
        rows, cols = np.asarray(rows), np.asarray(cols)
        w = (scaling_factors(band_sd(Y1), alpha)[rows] *
             scaling_factors(band_sd(Y2), alpha)[cols])
        phi = phi * w
        psi = psi * w
    return phi, psi
