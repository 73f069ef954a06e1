/*
 * oracle.c -- plain FP64 CPU oracle for generalized two-dimensional
 * correlation analysis (Geitner et al., "corr2D", arXiv 1808.00685).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP product path, and the product path
 * never calls it.
 *
 * Everything here is double precision and follows the paper's definitions
 * in their natural order: every sum runs over its index in increasing order,
 * with no blocking, reassociation or reuse beyond what the definition states.
 * OpenMP only distributes independent output rows over threads; it never
 * changes the order of any sum.
 *
 * Layouts: an input data matrix S holds m perturbation steps by rows and n
 * spectral points by columns, row-major with row stride ld (the paper's input
 * matrix convention, Sec. 3).  Full outputs are n1 x n2 row-major.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Dynamic spectra, Sec. 2 Eq. (dynspec) and Eq. (ref); Sec. 4.2 reference
 * spectrum code (column means when no reference is given, then subtraction
 * of the reference from every spectrum).
 *
 * Y[j*n + v] = S[j*ld + v] - r[v]      j = 0..m-1, v = 0..n-1
 * r = ref if ref != NULL, else r[v] = (1/m) * sum_j S[j*ld + v].
 * ref_out (may be NULL) receives r.                                          */
void oracle_dynamic(long m, long n, const double* S, long ld, const double* ref,
                    double* Y, double* ref_out)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (long v = 0; v < n; ++v) {
        if (ref) {
            r[v] = ref[v];
        } else {
            double s = 0.0;
            for (long j = 0; j < m; ++j) s += S[j * ld + v];
            r[v] = s / (double)m;
        }
    }
    for (long j = 0; j < m; ++j)
        for (long v = 0; v < n; ++v) Y[j * n + v] = S[j * ld + v] - r[v];
    if (ref_out)
        for (long v = 0; v < n; ++v) ref_out[v] = r[v];
    free(r);
}

/* Hilbert-Noda matrix, Sec. 2 Eq. (HilbNoda):
 * N[j][k] = 0 for j == k, 1/(pi (k - j)) otherwise; m x m row-major.        */
void oracle_hilbert_noda(long m, double* N)
{
    for (long j = 0; j < m; ++j)
        for (long k = 0; k < m; ++k)
            N[j * m + k] = (j == k) ? 0.0 : 1.0 / (M_PI * (double)(k - j));
}

/* Transpose helper for cache-friendly dot products.  It only moves values:
 * out[v*m + j] = in[j*n + v].                                               */
static double* columns_of(long m, long n, const double* in)
{
    double* out = (double*)malloc(sizeof(double) * (size_t)(m * n > 0 ? m * n : 1));
    for (long j = 0; j < m; ++j)
        for (long v = 0; v < n; ++v) out[v * m + j] = in[j * n + v];
    return out;
}

/* Hilbert transform of dynamic spectra by the Hilbert-Noda matrix,
 * Sec. 2 Eq. (disHT): Z[j][v] = sum_k N[j][k] * Y[k][v]  (k ascending).      */
void oracle_noda_transform(long m, long n, const double* Y, double* Z)
{
    double* N = (double*)malloc(sizeof(double) * (size_t)(m * m));
    oracle_hilbert_noda(m, N);
#pragma omp parallel for schedule(static)
    for (long v = 0; v < n; ++v) {
        for (long j = 0; j < m; ++j) {
            double s = 0.0;
            for (long k = 0; k < m; ++k) s += N[j * m + k] * Y[k * n + v];
            Z[j * n + v] = s;
        }
    }
    free(N);
}

/* Direct (Hilbert-transform) route, Sec. 2 Eqs. (disHTsyn), (disHT),
 * (HilbNoda), (disHTasyn):
 *   phi[a][b] = 1/(m-1) sum_j Y1[j][a] Y2[j][b]
 *   psi[a][b] = 1/(m-1) sum_j Y1[j][a] Z2[j][b],   Z2 = N Y2.
 * Y1: m x n1, Y2: m x n2 dynamic spectra (row-major).  Every entry of both
 * full n1 x n2 outputs is computed on its own (no mirroring), so symmetry
 * and antisymmetry of homocorrelation results are properties to be tested,
 * not assumptions.                                                           */
void oracle_corr_ht(long m, long n1, long n2, const double* Y1, const double* Y2,
                    double* phi, double* psi)
{
    double* Z2 = (double*)malloc(sizeof(double) * (size_t)(m * n2 > 0 ? m * n2 : 1));
    oracle_noda_transform(m, n2, Y2, Z2);
    double* c1 = columns_of(m, n1, Y1);
    double* c2 = columns_of(m, n2, Y2);
    double* cz = columns_of(m, n2, Z2);
    const double inv = 1.0 / (double)(m - 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < n1; ++a) {
        const double* ya = c1 + a * m;
        for (long b = 0; b < n2; ++b) {
            const double* yb = c2 + b * m;
            const double* zb = cz + b * m;
            double sp = 0.0, sq = 0.0;
            for (long j = 0; j < m; ++j) {
                sp += ya[j] * yb[j];
                sq += ya[j] * zb[j];
            }
            phi[a * n2 + b] = sp * inv;
            psi[a * n2 + b] = sq * inv;
        }
    }
    free(c1);
    free(c2);
    free(cz);
    free(Z2);
}

/* Selected entries of the direct route (for spot checks of outputs too large
 * to compute in full).  For each t < count: rows[t] indexes Y1's columns,
 * cols[t] indexes Y2's columns; same formulas as oracle_corr_ht.             */
void oracle_corr_ht_entries(long m, long n1, long n2, const double* Y1, const double* Y2,
                            long count, const long* rows, const long* cols,
                            double* phi, double* psi)
{
    double* N = (double*)malloc(sizeof(double) * (size_t)(m * m));
    oracle_hilbert_noda(m, N);
    const double inv = 1.0 / (double)(m - 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < count; ++t) {
        const long a = rows[t], b = cols[t];
        double sp = 0.0, sq = 0.0;
        for (long j = 0; j < m; ++j) {
            double z = 0.0; /* Z2[j][b] = sum_k N[j][k] Y2[k][b] */
            for (long k = 0; k < m; ++k) z += N[j * m + k] * Y2[k * n2 + b];
            sp += Y1[j * n1 + a] * Y2[j * n2 + b];
            sq += Y1[j * n1 + a] * z;
        }
        phi[t] = sp * inv;
        psi[t] = sq * inv;
    }
    (void)n1;
    free(N);
}

/* Discrete Fourier transform along the perturbation axis, Sec. 2 Eq. (disFT):
 *   F[w][v] = sum_{j=0}^{m-1} Y[j][v] exp(-2 pi i w j / m),  w = 0..m-1
 * (the paper's j = 1..m with exponent (j-1)).  Direct O(m^2) evaluation; the
 * phase w*j is reduced modulo m exactly before the trigonometric call.
 * Output re/im: m x n row-major.                                             */
void oracle_dft(long m, long n, const double* Y, double* re, double* im)
{
#pragma omp parallel for schedule(static)
    for (long v = 0; v < n; ++v) {
        for (long w = 0; w < m; ++w) {
            double sr = 0.0, si = 0.0;
            for (long j = 0; j < m; ++j) {
                const long ph = (w * j) % m;
                const double ang = 2.0 * M_PI * (double)ph / (double)m;
                sr += Y[j * n + v] * cos(ang);
                si -= Y[j * n + v] * sin(ang);
            }
            re[w * n + v] = sr;
            im[w * n + v] = si;
        }
    }
}

/* Fourier-transform route with the m-point DFT (Sec. 2 Eqs. (disFT),
 * (disint2d), (symmeFT); Sec. 4.2: only one half of the spectrum is used and
 * every bin except DC is counted twice).  Reading: the half spectrum is
 * Hermitian-complete -- DC weight 1, bins 0 < w < m/2 weight 2, the Nyquist
 * bin w = m/2 (even m) weight 1 -- so that the weighted half sum equals the
 * full-spectrum sum for the real part.
 *   C[a][b] = cF * sum_{w in half} weight(w) F1(w)[a] conj(F2(w)[b])
 *   phi = Re C, psi = Im C.
 * cF is the normalization applied to the Fourier sum: 1/(pi (m-1)) is the
 * paper's default Norm (Sec. 4.2); 1/(m (m-1)) reproduces the direct route's
 * synchronous spectrum (Parseval).                                           */
void oracle_corr_ft_circular(long m, long n1, long n2, const double* Y1, const double* Y2,
                             double cF, double* phi, double* psi)
{
    double* r1 = (double*)malloc(sizeof(double) * (size_t)(m * n1));
    double* i1 = (double*)malloc(sizeof(double) * (size_t)(m * n1));
    double* r2 = (double*)malloc(sizeof(double) * (size_t)(m * n2));
    double* i2 = (double*)malloc(sizeof(double) * (size_t)(m * n2));
    oracle_dft(m, n1, Y1, r1, i1);
    oracle_dft(m, n2, Y2, r2, i2);
    const long half = m / 2; /* bins 0..half */
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < n1; ++a) {
        for (long b = 0; b < n2; ++b) {
            double sr = 0.0, si = 0.0;
            for (long w = 0; w <= half; ++w) {
                double wt = 2.0;
                if (w == 0 || (2 * w == m)) wt = 1.0;
                /* F1 conj(F2) = (x1 + i y1)(x2 - i y2) */
                const double x1 = r1[w * n1 + a], y1 = i1[w * n1 + a];
                const double x2 = r2[w * n2 + b], y2 = i2[w * n2 + b];
                sr += wt * (x1 * x2 + y1 * y2);
                si += wt * (y1 * x2 - x1 * y2);
            }
            phi[a * n2 + b] = cF * sr;
            psi[a * n2 + b] = cF * si;
        }
    }
    free(r1);
    free(i1);
    free(r2);
    free(i2);
}

/* Zero-padded Fourier route that reproduces the direct (Hilbert-Noda) route
 * exactly.  Both dynamic spectra are zero-padded to L >= 2m-1 points (the
 * "0 outside the perturbation interval" of Eq. (dynspec)) and transformed by
 * an L-point DFT.  Then, with G(w) = F1(w) conj(F2(w)),
 *   phi + i psi = 1/(L (m-1)) sum_{w=0}^{L-1} G(w) (1 + tau(w)),
 *   tau(w) = (2/pi) sum_{d=1}^{m-1} sin(2 pi w d / L) / d.
 * Derivation: with padding, (1/L) sum_w G(w) exp(2 pi i w d / L) is the
 * non-circular lag-d cross product sum_j y1[j + d] y2[j]; weighting the lags
 * d != 0 by the Hilbert-Noda kernel 1/(pi d) gives the sine series tau.  This
 * is an independent algorithm for the same result, used to pin the direct
 * route ("FT and HT agree", Sec. 2).                                         */
void oracle_corr_ft_padded(long m, long n1, long n2, const double* Y1, const double* Y2,
                           long L, double* phi, double* psi)
{
    double* tau = (double*)malloc(sizeof(double) * (size_t)L);
    for (long w = 0; w < L; ++w) {
        double s = 0.0;
        for (long d = 1; d <= m - 1; ++d) {
            const long ph = (w * d) % L;
            s += sin(2.0 * M_PI * (double)ph / (double)L) / (double)d;
        }
        tau[w] = 2.0 / M_PI * s;
    }
    double* P1 = (double*)calloc((size_t)(L * n1), sizeof(double));
    double* P2 = (double*)calloc((size_t)(L * n2), sizeof(double));
    memcpy(P1, Y1, sizeof(double) * (size_t)(m * n1));
    memcpy(P2, Y2, sizeof(double) * (size_t)(m * n2));
    double* r1 = (double*)malloc(sizeof(double) * (size_t)(L * n1));
    double* i1 = (double*)malloc(sizeof(double) * (size_t)(L * n1));
    double* r2 = (double*)malloc(sizeof(double) * (size_t)(L * n2));
    double* i2 = (double*)malloc(sizeof(double) * (size_t)(L * n2));
    oracle_dft(L, n1, P1, r1, i1);
    oracle_dft(L, n2, P2, r2, i2);
    const double norm = 1.0 / ((double)L * (double)(m - 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < n1; ++a) {
        for (long b = 0; b < n2; ++b) {
            double sr = 0.0, si = 0.0;
            for (long w = 0; w < L; ++w) {
                const double x1 = r1[w * n1 + a], y1 = i1[w * n1 + a];
                const double x2 = r2[w * n2 + b], y2 = i2[w * n2 + b];
                const double gr = x1 * x2 + y1 * y2, gi = y1 * x2 - x1 * y2;
                sr += gr * (1.0 + tau[w]);
                si += gi * (1.0 + tau[w]);
            }
            phi[a * n2 + b] = norm * sr;
            psi[a * n2 + b] = norm * si;
        }
    }
    free(tau);
    free(P1);
    free(P2);
    free(r1);
    free(i1);
    free(r2);
    free(i2);
}

/* Selected entries of the m-point circular Fourier route (same definition as
 * oracle_corr_ft_circular), for spot checks at large n.  Each entry evaluates
 * the two needed DFT columns directly.                                       */
void oracle_corr_ft_circular_entries(long m, long n1, long n2, const double* Y1,
                                     const double* Y2, double cF, long count,
                                     const long* rows, const long* cols,
                                     double* phi, double* psi)
{
    const long half = m / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < count; ++t) {
        const long a = rows[t], b = cols[t];
        double sr = 0.0, si = 0.0;
        for (long w = 0; w <= half; ++w) {
            double x1 = 0.0, y1 = 0.0, x2 = 0.0, y2 = 0.0;
            for (long j = 0; j < m; ++j) {
                const long ph = (w * j) % m;
                const double ang = 2.0 * M_PI * (double)ph / (double)m;
                x1 += Y1[j * n1 + a] * cos(ang);
                y1 -= Y1[j * n1 + a] * sin(ang);
                x2 += Y2[j * n2 + b] * cos(ang);
                y2 -= Y2[j * n2 + b] * sin(ang);
            }
            double wt = 2.0;
            if (w == 0 || (2 * w == m)) wt = 1.0;
            sr += wt * (x1 * x2 + y1 * y2);
            si += wt * (y1 * x2 - x1 * y2);
        }
        phi[t] = cF * sr;
        psi[t] = cF * si;
    }
}

/* Number of OpenMP threads the parallel loops above use (reported with the
 * CPU-baseline timing).                                                      */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops of later calls (at least 1); the CPU
 * baseline times some sizes on one thread.                                   */
void oracle_set_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}
