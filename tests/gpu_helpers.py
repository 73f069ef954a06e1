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
TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-5, "split_f16": 1e-5, "bf16": 2 * 2.0 ** -8,
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
# split-FP16: halves of 11 bits after the per-band scale (u = 2^-11), so the
# products err by at most 3 u^2 |a||b| = 3 2^-22 |a||b|; the FP32
# accumulation and transform dominate, as for FP32 (2^-14).
ELEMENT_TAU = {"split_bf16": 2.0 ** -13, "f32": 2.0 ** -14, "bf16": 2.0 ** -6, "f64": 2.0 ** -40,
               "f16": 2.0 ** -9, "fp8_e4m3": 2.0 ** -2, "split_f16": 2.0 ** -14}


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


# ---------------------------------------------------------------------------
# Full-matrix comparisons of outputs too large to hold twice in FP64.  The
# arithmetic of the comparison runs in torch (FP64) on the device that holds
# the oracle's blocks; the oracle's values themselves come from oracle/.
# ---------------------------------------------------------------------------
class FullError:
    """Relative Frobenius errors ||G - O||_F / ||O||_F of Phi and Psi over the
    full matrices, accumulated block by block, and the largest ratio of an
    entry's error to its per-element bound (ELEMENT_TAU) seen.  For a
    homocorrelation given as upper-triangle rows, each entry off the
    diagonal stands for two entries of the full matrix (Phi symmetric, Psi
    antisymmetric), so it counts twice; `diag` indexes the diagonal entries
    of the block, which count once."""

    def __init__(self):
        self.num = [0.0, 0.0]
        self.den = [0.0, 0.0]
        self.bound_ratio = 0.0
        self.entries = 0

    def add(self, k, g, o, diag=None, bound=None):
        import torch
        g = g.to(device=o.device, dtype=torch.float64)
        d = g - o
        d2, o2 = d * d, o * o
        if diag is None:
            self.num[k] += float(d2.sum())
            self.den[k] += float(o2.sum())
        else:
            self.num[k] += float(2.0 * d2.sum() - d2[diag].sum())
            self.den[k] += float(2.0 * o2.sum() - o2[diag].sum())
        if bound is not None:
            err = d.abs()
            zero_b = bound <= 0
            # an entry whose bound is zero (a zero dynamic spectrum) must be exact
            if bool(torch.any(err[zero_b] > 0)):
                self.bound_ratio = float("inf")
            r = torch.where(zero_b, torch.zeros_like(err), err / torch.where(zero_b, torch.ones_like(bound), bound))
            if r.numel():
                self.bound_ratio = max(self.bound_ratio, float(r.max()))
        if k == 0:
            self.entries += int(g.numel())

    def rel(self, k):
        if self.den[k] == 0:
            return float(np.sqrt(self.num[k]))
        return float(np.sqrt(self.num[k] / self.den[k]))


def packed_rows(plane, n, r0, r1, base=0):
    """Rows r0..r1-1 of an UPPER_PACKED plane (a torch tensor), in packed
    order (row i: columns i..n-1), on the plane's device."""
    s = base + r0 * n - (r0 * (r0 - 1)) // 2
    e = base + r1 * n - (r1 * (r1 - 1)) // 2
    return plane[s:e]


def aligned_rows(plane, n, r0, r1):
    """Rows r0..r1-1 of an UPPER_ALIGNED plane gathered into packed order on
    the plane's device.  Index of (i, j) from the layout's definition:
    i N32 - 32 (16 q (q-1) + r q) + (j - 32 q), i = 32 q + r."""
    import torch
    dev = plane.device
    i = torch.arange(r0, r1, device=dev, dtype=torch.int64)
    lens = n - i
    rows = torch.repeat_interleave(i, lens)
    start = torch.cumsum(lens, 0) - lens
    j = torch.arange(rows.numel(), device=dev, dtype=torch.int64) - start[rows - r0] + rows
    n32 = (n + 31) // 32 * 32
    q, r = rows // 32, rows % 32
    idx = rows * n32 - 32 * (16 * q * (q - 1) + r * q) + (j - 32 * q)
    return plane[idx]


def oracle_upper_blocks(oracle, S, device, block=1024, alpha=0.0):
    """The oracle's homocorrelation (Noda's kernel and norm) as upper-triangle
    row blocks in packed order, moved to `device` as FP64 torch tensors: list
    of (r0, r1, phi, psi, diag, bphi, bpsi), diag the positions of the
    diagonal entries, b* the per-element bound factors ||y_i|| ||y_j|| / (m-1)
    (Phi) and ||y_i|| ||(N y)_j|| / (m-1) (Psi) that ELEMENT_TAU multiplies.
    alpha scales as oracle.corr2d does."""
    import torch
    Y, _ = oracle.dynamic(S)
    m, n = Y.shape
    ny = np.linalg.norm(Y, axis=0)
    nz = np.linalg.norm(oracle.noda_transform(Y), axis=0)
    f = oracle.scaling_factors(oracle.band_sd(Y), alpha) if alpha else None
    out = []
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=device)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        po, qo = oracle.corr_ht_block(Y, Y, r0, r1, r0, n)
        mask = np.triu(np.ones((r1 - r0, n - r0), dtype=bool))
        bp = np.outer(ny[r0:r1], ny[r0:]) / (m - 1)
        bq = np.outer(ny[r0:r1], nz[r0:]) / (m - 1)
        if f is not None:
            w = np.outer(f[r0:r1], f[r0:])
            po, qo, bp, bq = po * w, qo * w, bp * w, bq * w
        l = np.arange(r1 - r0, dtype=np.int64)
        diag = l * (n - r0) - (l * (l - 1)) // 2
        out.append((r0, r1, t(po[mask]), t(qo[mask]), t(diag), t(bp[mask]), t(bq[mask])))
        del po, qo, bp, bq, mask
    return out


def homo_full_error(blocks, get_rows, tau=None):
    """FullError of a GPU homocorrelation against oracle_upper_blocks(...);
    get_rows(k, r0, r1) returns rows r0..r1-1 of plane k (0 Phi, 1 Psi) in
    packed order."""
    fe = FullError()
    for r0, r1, po, qo, diag, bp, bq in blocks:
        for k, (o, b) in enumerate(((po, bp), (qo, bq))):
            g = get_rows(k, r0, r1)
            assert g.numel() == o.numel(), (g.numel(), o.numel())
            fe.add(k, g, o, diag, None if tau is None else tau * b)
    return fe
