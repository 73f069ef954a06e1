"""Helpers shared by the GPU parity tests (comparison and unpacking only)."""
import numpy as np

# Tolerances on the relative Frobenius error ||G - O||_F / ||O||_F, per output
# (Phi and Psi separately).  F64, F32 and split-BF16 follow the stated
# targets.  For the single-rounding formats the bound is derived from the unit
# roundoff u (BF16 2^-8, FP16 2^-11, FP8 e4m3 2^-4): each product of two
# rounded operands carries a relative error below 2u, so an output whose
# terms do not cancel has relative error below 2u; random test data (whose
# off-diagonal sums do cancel) measures about 0.6u.  The stricter 2e-3 target
# of plain BF16 applies to the band workload (BF16_BAND_TOL).
TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-5, "bf16": 2 * 2.0 ** -8,
       "f16": 2 * 2.0 ** -11, "fp8_e4m3": 2 * 2.0 ** -4}
BF16_BAND_TOL = 2e-3

# Per-element bound factors tau: |err_ij| <= tau ||y_i|| ||(N y)_j|| / (m-1)
# for Psi (||y_j|| for Phi), in either basis (Fourier: c = 1/(m(m-1)) and
# ||a_i|| = sqrt(m) ||y_i|| by Parseval; time: c = 1/(m-1), a = y, b = N y),
# through sum|a_k||b_k| <= ||a|| ||b||.
# split-BF16: with unit roundoff u = 2^-8 of BF16, |x - hi| <= u|x| and lo
# carries u|lo| <= u^2|x|, so the products err by at most 3 u^2 |a||b|
# (lo.lo dropped, lo rounded), FP32 accumulation of 3K products by
# 3K 2^-24 sum|a||b| (4.6e-5 at K = 256), the FP32 transform by ~1e-6;
# FP32: operands rounded by 2^-24, K-term FP32 accumulation and the FP32
# transform (each <= 1.5e-5 worst case at K = 256); BF16: operands rounded by
# u, products by 2u + u^2, plus accumulation; FP16 (u = 2^-11) and FP8 e4m3
# (u = 2^-4) the same, per-band scaling putting each column's largest values
# near the top of the format's range, so that subnormal errors are
# negligible against the column norms; FP64: the FP64 transform and
# accumulation.
ELEMENT_TAU = {"split_bf16": 2.0 ** -13, "f32": 2.0 ** -14, "bf16": 2.0 ** -6, "f64": 2.0 ** -40,
               "f16": 2.0 ** -9, "fp8_e4m3": 2.0 ** -2}


def rel_fro(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    den = np.linalg.norm(o)
    if den == 0:
        return float(np.linalg.norm(g))
    return float(np.linalg.norm(g - o) / den)


def unpack_upper(p, n):
    """Full matrices from the UPPER_PACKED layout (row i holds j = i..n-1)."""
    p = np.asarray(p)
    full = np.zeros((n, n), dtype=p.dtype)
    off = 0
    for i in range(n):
        full[i, i:] = p[off:off + n - i]
        off += n - i
    return full


def aligned_row_starts(n):
    """Row starts of the UPPER_ALIGNED layout from its definition: row i holds
    the columns 32 floor(i/32) .. N32-1 (N32 = n rounded up to 32), rows stored
    one after another.  Returns (starts with the total appended, first columns)."""
    n32 = -(-n // 32) * 32
    first = 32 * (np.arange(n, dtype=np.int64) // 32)
    lens = n32 - first
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), first


def unpack_upper_aligned(p, n):
    """Upper-triangle matrices (zeros below) and the mask of padding slots
    from an UPPER_ALIGNED plane."""
    p = np.asarray(p)
    starts, first = aligned_row_starts(n)
    full = np.zeros((n, n), dtype=p.dtype)
    pad = np.ones(len(p), dtype=bool)
    for i in range(n):
        a = starts[i] + (i - first[i])
        full[i, i:] = p[a:a + n - i]
        pad[a:a + n - i] = False
    return full, pad


def packed_index(i, j, n):
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * n - (i * (i - 1)) // 2 + (j - i)


def check_homo_structure(phi, psi):
    """Exact mirror structure of a FULL homocorrelation output."""
    assert np.array_equal(phi, phi.T)
    assert np.array_equal(psi, -psi.T)
    assert np.all(np.diag(psi) == 0)
