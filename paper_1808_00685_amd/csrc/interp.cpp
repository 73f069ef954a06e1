// interp.cpp -- weights of the interpolation to equidistant perturbation
// values (Sec. 4.1): the target grid is T_k = t_0 + k (t_last - t_0)/(N-1),
// k = 0..N-1, and each spectral variable is interpolated along t either
// piecewise linearly or with the cubic spline of Forsythe, Malcolm and Moler
// (end third derivatives equal to those of the cubics through the first and
// the last four points; three points give the parabola, two the line).
//
// Both are linear in the data, so the resampled spectra are W y with an
// N x m_in matrix W, built here once per plan in FP64: column i of W is the
// interpolant of the unit vector e_i evaluated on the target grid.
#include "interp.h"

#include <cmath>

namespace corr2d {
namespace {

// Second derivatives M of the FMM spline through (x, y): interior rows of
// the usual tridiagonal system, the end conditions (M1 - M0)/h0 = tl and
// (M[n-1] - M[n-2])/h[n-2] = tr eliminated into the first and last interior
// rows, then the Thomas algorithm (the reduced system is diagonally
// dominant).
void fmm_second_derivatives(const std::vector<double>& x, const std::vector<double>& y,
                            std::vector<double>& M) {
    const size_t n = x.size();
    M.assign(n, 0.0);
    if (n < 3) return;
    std::vector<double> h(n - 1), d(n - 1);
    for (size_t i = 0; i + 1 < n; ++i) {
        h[i] = x[i + 1] - x[i];
        d[i] = (y[i + 1] - y[i]) / h[i];
    }
    if (n == 3) {
        // zero third derivative at both ends: one parabola, M = 2 f[x0,x1,x2]
        const double m = 2.0 * (d[1] - d[0]) / (h[0] + h[1]);
        M[0] = M[1] = M[2] = m;
        return;
    }
    // 6 x third divided difference of four consecutive points
    auto third = [&](size_t s) {
        const double d20 = (d[s + 1] - d[s]) / (x[s + 2] - x[s]);
        const double d21 = (d[s + 2] - d[s + 1]) / (x[s + 3] - x[s + 1]);
        return 6.0 * (d21 - d20) / (x[s + 3] - x[s]);
    };
    const double tl = third(0), tr = third(n - 4);
    const size_t k = n - 2;   // unknowns M1..M[n-2]
    std::vector<double> a(k), b(k), c(k), r(k);
    for (size_t j = 0; j < k; ++j) {
        const size_t i = j + 1;
        a[j] = h[i - 1];
        b[j] = 2.0 * (h[i - 1] + h[i]);
        c[j] = h[i];
        r[j] = 6.0 * (d[i] - d[i - 1]);
    }
    // M0 = M1 - h0 tl into the first row, M[n-1] = M[n-2] + h[n-2] tr into
    // the last
    b[0] += h[0];
    r[0] += h[0] * h[0] * tl;
    b[k - 1] += h[n - 2];
    r[k - 1] -= h[n - 2] * h[n - 2] * tr;
    for (size_t j = 1; j < k; ++j) {
        const double w = a[j] / b[j - 1];
        b[j] -= w * c[j - 1];
        r[j] -= w * r[j - 1];
    }
    std::vector<double> s(k);
    s[k - 1] = r[k - 1] / b[k - 1];
    for (size_t j = k - 1; j-- > 0;) s[j] = (r[j] - c[j] * s[j + 1]) / b[j];
    for (size_t j = 0; j < k; ++j) M[j + 1] = s[j];
    M[0] = M[1] - h[0] * tl;
    M[n - 1] = M[n - 2] + h[n - 2] * tr;
}

// Interval [x_i, x_{i+1}] of t (t inside [x_0, x_last]).
size_t interval(const std::vector<double>& x, double t) {
    size_t lo = 0, hi = x.size() - 1;
    while (hi - lo > 1) {
        const size_t mid = (lo + hi) / 2;
        if (x[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace

bool build_interp_weights(const double* t_in, int64_t m_in, int64_t N, int method, InterpWeights& w) {
    w.m_in = m_in;
    w.N = N;
    w.W.assign((size_t)(N * m_in), 0.0);
    std::vector<double> x(t_in, t_in + m_in);
    std::vector<double> T((size_t)N);
    const double t0 = x.front(), t1 = x.back();
    for (int64_t k = 0; k < N; ++k)
        T[(size_t)k] = (k == N - 1) ? t1 : t0 + (t1 - t0) * (double)k / (double)(N - 1);
    if (method == 1 || m_in == 2) {
        // piecewise linear (also the spline of two points)
        for (int64_t k = 0; k < N; ++k) {
            const size_t i = interval(x, T[(size_t)k]);
            const double u = (T[(size_t)k] - x[i]) / (x[i + 1] - x[i]);
            w.W[(size_t)k * m_in + i] += 1.0 - u;
            w.W[(size_t)k * m_in + i + 1] += u;
        }
    } else {
        std::vector<double> e((size_t)m_in, 0.0), M;
        for (int64_t i = 0; i < m_in; ++i) {
            e[(size_t)i] = 1.0;
            fmm_second_derivatives(x, e, M);
            for (int64_t k = 0; k < N; ++k) {
                const double t = T[(size_t)k];
                const size_t j = interval(x, t);
                const double h = x[j + 1] - x[j], a = x[j + 1] - t, b = t - x[j];
                const double v = M[j] * a * a * a / (6.0 * h) + M[j + 1] * b * b * b / (6.0 * h) +
                                 (e[j] / h - M[j] * h / 6.0) * a + (e[j + 1] / h - M[j + 1] * h / 6.0) * b;
                w.W[(size_t)k * m_in + i] = v;
            }
            e[(size_t)i] = 0.0;
        }
    }
    // nonzero input rows of each block of kInterpRows output rows
    const int64_t nb = (N + kInterpRows - 1) / kInterpRows;
    w.block_range.assign((size_t)(2 * nb), 0);
    for (int64_t blk = 0; blk < nb; ++blk) {
        int64_t lo = m_in, hi = 0;
        for (int64_t k = blk * kInterpRows; k < N && k < (blk + 1) * kInterpRows; ++k)
            for (int64_t i = 0; i < m_in; ++i)
                if (w.W[(size_t)(k * m_in + i)] != 0.0) {
                    lo = i < lo ? i : lo;
                    hi = i + 1 > hi ? i + 1 : hi;
                }
        if (lo >= hi) lo = hi = 0;
        w.block_range[(size_t)(2 * blk)] = (int32_t)lo;
        w.block_range[(size_t)(2 * blk + 1)] = (int32_t)hi;
    }
    for (double v : w.W)
        if (!std::isfinite(v)) return false;
    return true;
}

}  // namespace corr2d
