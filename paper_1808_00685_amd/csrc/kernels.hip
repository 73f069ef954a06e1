// kernels.hip -- HIP kernels (gfx950 / CDNA4) of the correlation hot path.
//
// Pipeline of one call (Geitner et al., arXiv 1808.00685, Sec. 2 and 4.2):
//   tables_kernel     the m x m transforms: T1 = real-packed Hermitian half
//                     spectrum DFT (Eqs. (disFT), (symmeFT)), T2 = the
//                     asynchronous operand's transform (T1 N for Noda's
//                     kernel, Eq. (HilbNoda); a row-pair rotation of T1 for
//                     the circular kernel).
//   center_kernel     FP64 perturbation mean and dynamic spectra
//                     (Eqs. (dynspec), (ref)), transposed so that each
//                     spectral point's m values are contiguous; per-band
//                     power-of-two scales from the column norm.
//   transform_kernel, transform32_kernel
//                     MFMA GEMM  [A | B] = Yc^T [T1 | T2]^T  (FP64, or FP32
//                     for the reduced formats); the epilogue scales, rounds
//                     (RNE) and packs the contraction operands, zero padded
//                     (panel-blocked for the 16-bit formats).
//   center_transform32_kernel
//                     the centring and transform32_kernel in one kernel for
//                     m up to 256 (all formats but FP64): each workgroup
//                     centres its 64 spectral points into LDS and multiplies
//                     them by the tables there, no centred spectra in HBM.
//   fft_tables_kernel, fft_transform_kernel
//                     for power-of-two m in [128, 1024] (FP64 for the FP64
//                     path, else FP32) in place of the three kernels above: twiddles and the
//                     Noda multiplier, then per workgroup the centring (FP64)
//                     fused with radix FFTs in LDS that produce the same
//                     packed operands (A from the spectra, Noda's B through
//                     an FFT correlation).
//   corr2_kernel, corr_kernel
//                     MFMA GEMM over output tiles: Phi = c A1^T A2,
//                     Psi = c A1^T B2 (Eq. (disint2d) evaluated as a real
//                     contraction over the packed half spectrum), FP64
//                     epilogue, upper-triangle tiles for homocorrelation with
//                     exact mirror or upper-triangle stores (LDS-staged ring
//                     and 32x32 MFMA for the 16-bit formats, register-direct
//                     16x16 MFMA for FP64, FP32 and FP8).
//   interp_kernel     resampling onto equidistant perturbation values
//                     (Sec. 4.1) ahead of the centring, when asked for.
//
// MFMA fragment convention (16x16 family): lane l supplies row (l & 15) and
// the contraction slice (l >> 4) of its operand; the accumulator register q
// of lane l holds column (l & 15) and row 4*(l >> 4) + q for the FP32-output
// instructions, but row (l >> 4) + 4*q for v_mfma_f64_16x16x4f64 (measured).
#include <hip/hip_runtime.h>
#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "corr2d_internal.h"
#include "launch.h"
#include "tile_order.h"

namespace corr2d {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ rounding
// Two floats -> a packed pair of bfloat16 (a in the low half), round to
// nearest even: v_cvt_pk_bf16_f32.
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ inline uint32_t bf16x2_rne(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2v));
}
// Split of a pair: hi = RNE(x), lo = RNE(x - hi) (x - hi is exact in FP32).
__device__ inline void bf16x2_split(float a, float b, uint32_t& hi, uint32_t& lo) {
    hi = bf16x2_rne(a, b);
    lo = bf16x2_rne(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

// Split of four floats into FP16 halves: hi = RNE(x), lo = RNE(x - hi) (x - hi
// is exact in FP32 while |x| stays within the FP16 range, which the per-band
// scales guarantee).
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
__device__ inline void f16x4_split(const float* x, h4v& hi, h4v& lo) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        hi[q] = (_Float16)x[q];
        lo[q] = (_Float16)(x[q] - (float)hi[q]);
    }
}

// float -> OCP FP8 e4m3 (bias 7, 3 mantissa bits, largest finite 448, no
// infinities), round to nearest even, saturating at +-448; NaN -> 0x7f.
__device__ inline uint8_t fp8_e4m3_rne(float x) {
    if (x != x) return 0x7f;
    const uint8_t sgn = (__float_as_uint(x) >> 31) ? 0x80 : 0x00;
    float a = fabsf(x);
    if (a >= 480.0f) return sgn | 0x7e;
    uint32_t code;
    if (a < 0.015625f) {                      // below 2^-6: subnormal grid 2^-9
        code = (uint32_t)rintf(a * 512.0f);    // 0..8; 8 is the smallest normal
    } else {
        int e;
        float f = frexpf(a, &e);              // a = f 2^e, f in [0.5, 1)
        float mant = f * 2.0f;                // [1, 2)
        int ex = e - 1;
        uint32_t q = (uint32_t)rintf((mant - 1.0f) * 8.0f);
        if (q == 8) { q = 0; ++ex; }
        code = (uint32_t)((ex + 7) << 3) | q;
    }
    if (code >= 0x7f) code = 0x7e;            // 0x7f is NaN: saturate to 448
    return sgn | (uint8_t)code;
}

// ------------------------------------------------------------ XCD placement
// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD receives one contiguous run of the tile order (its L2 then holds the
// operand panels that run shares).
// A value known to be equal in all lanes, moved to scalar registers.
__device__ inline int64_t uniform64(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t per = nb / 8, rem = nb % 8;
    const int64_t x = b % 8, s = b / 8;
    return x * per + (x < rem ? x : rem) + s;
}

// =========================================================================
// Transform tables
// =========================================================================
struct TwiddleView {
    const double* c;
    const double* s;
    int64_t m;
};

// Row r of the real-packed Fourier basis at time index l: row 0 is DC, rows
// 2p-1 / 2p carry sqrt2 Re / sqrt2 Im of exp(-2 pi i p l / m) for
// 0 < p < m/2, and row m-1 of an even m is the Nyquist bin.  With this
// packing the weighted half-spectrum sum of Eq. (symmeFT) is a plain dot
// product of rows, and Q^T Q = m I.
__device__ inline double qrow(const TwiddleView tw, int64_t r, int64_t l) {
    const int64_t m = tw.m;
    if (r == 0) return 1.0;
    if ((m & 1) == 0 && r == m - 1) return (l & 1) ? -1.0 : 1.0;
    const int64_t p = (r + 1) >> 1;
    const int64_t idx = (p * l) % m;
    return (r & 1) ? M_SQRT2 * tw.c[idx] : -M_SQRT2 * tw.s[idx];
}

// Row r of J Q: each (Re, Im) pair becomes (-Im, Re); DC and Nyquist vanish.
// A1^T (J A2) is then the imaginary part of the weighted sum of
// F1 conj(F2) -- the circular asynchronous kernel of the m-point route.
__device__ inline double jqrow(const TwiddleView tw, int64_t r, int64_t l) {
    const int64_t m = tw.m;
    if (r == 0) return 0.0;
    if ((m & 1) == 0 && r == m - 1) return 0.0;
    const int64_t p = (r + 1) >> 1;
    const int64_t idx = (p * l) % m;
    return (r & 1) ? M_SQRT2 * tw.s[idx] : M_SQRT2 * tw.c[idx];
}

// sum_{l != j} Q[k][l] / (pi (j - l)) with h[d + m] = 1/(pi d) from LDS and
// the twiddle index p*l mod m advanced incrementally.
__device__ inline double qn_entry(const TwiddleView tw, const double* h, int64_t k, int64_t j) {
    const int64_t m = tw.m;
    if (k == 0) {
        double s = 0.0;
        for (int64_t l = 0; l < m; ++l)
            if (l != j) s += h[j - l + m];
        return s;
    }
    if ((m & 1) == 0 && k == m - 1) {
        double s = 0.0;
        for (int64_t l = 0; l < m; ++l)
            if (l != j) s += ((l & 1) ? -1.0 : 1.0) * h[j - l + m];
        return s;
    }
    const int64_t p = (k + 1) >> 1;
    const double* t = (k & 1) ? tw.c : tw.s;
    const double sg = (k & 1) ? M_SQRT2 : -M_SQRT2;
    double s = 0.0;
    int64_t idx = 0;
    for (int64_t l = 0; l < m; ++l) {
        if (l != j) s += t[idx] * h[j - l + m];
        idx += p;
        if (idx >= m) idx -= m;
    }
    return sg * s;
}

// Row factor of the R code's bin list (Sec. 4.2: bins floor(j/2) for
// j = 1..m-1) relative to the Hermitian-complete packing: the pair of the top
// bin (m-1)/2 of an odd m counts once instead of twice (1/sqrt2 on both of
// its rows), the Nyquist row of an even m not at all.
__device__ inline double r_compat_row(int64_t m, int64_t r) {
    if ((m & 1) == 0) return r == m - 1 ? 0.0 : 1.0;
    return (m > 1 && (r == m - 2 || r == m - 1)) ? M_SQRT1_2 : 1.0;
}

__device__ inline double table_entry(const TableJob& T, const TwiddleView tw, const double* h,
                                     int64_t r, int64_t j) {
    const int64_t m = T.m;
    if (j >= m) return 0.0;
    if (r < T.kp) {
        if (r >= m) return 0.0;
        if (T.hilbert == H_R_COMPAT) return qrow(tw, r, j) * r_compat_row(m, r);
        return T.basis == B_FOURIER ? qrow(tw, r, j) : (r == j ? 1.0 : 0.0);
    }
    const int64_t k = r - T.kp;
    if (k >= m || r >= 2 * (int64_t)T.kp) return 0.0;
    if (T.basis == B_FOURIER) {
        if (T.hilbert == H_R_COMPAT) return jqrow(tw, k, j) * r_compat_row(m, k);
        if (T.hilbert == H_CIRCULAR) return jqrow(tw, k, j);
        // (Q N)[k][j] = sum_{l != j} Q[k][l] / (pi (j - l))
        return qn_entry(tw, h, k, j);
    }
    if (T.hilbert == H_NODA) return k == j ? 0.0 : h[j - k + m];
    // circular kernel in the time basis: (1/m) sum_r Q[r][k] (J Q)[r][j]
    double s = 0.0;
    for (int64_t q = 0; q < m; ++q) s += qrow(tw, q, k) * jqrow(tw, q, j);
    return s / (double)m;
}

constexpr int kMaxTwiddle = 4096;

// Dynamic LDS: cos and sin of 2 pi i / m (m entries each), then
// hh[d + m] = 1/(pi d) for -m < d < m (2m entries); 32 m bytes in all.
template <class Src>
__device__ inline void tables_body(const Src& src, int blk, double* tw_lds) {
    int lb;
    const TableJob T = src.get(blk, lb);
    double* tc = tw_lds;
    double* ts = tw_lds + T.m;
    double* hh = tw_lds + 2 * T.m;
    if (blk == 0 && src.counter && (int)threadIdx.x < src.ncounters) src.counter[threadIdx.x] = 0;
    for (int64_t i = threadIdx.x; i < T.m; i += blockDim.x) {
        double sv, cv;
        sincospi(2.0 * (double)i / (double)T.m, &sv, &cv);
        tc[i] = cv;
        ts[i] = sv;
    }
    for (int64_t d = (int64_t)threadIdx.x - T.m; d < T.m; d += blockDim.x)
        hh[d + T.m] = d == 0 ? 0.0 : 1.0 / (M_PI * (double)d);
    __syncthreads();
    const TwiddleView tw{tc, ts, T.m};
    const int64_t e = (int64_t)lb * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)T.rows_pad * T.kt;
    if (e >= total) return;
    const int64_t r = e / T.kt, j = e % T.kt;
    // the rows of Q N (Fourier basis, Noda's kernel) come from tables_qn_kernel
    if (T.basis == B_FOURIER && T.hilbert == H_NODA && r >= T.kp && r < T.kp + T.m && j < T.m) return;
    const double v = table_entry(T, tw, hh, r, j);
    if (T.f64) ((double*)T.table)[e] = v;
    else ((float*)T.table)[e] = (float)v;
}

template <class Src>
__global__ __launch_bounds__(256) void tables_kernel(Src src) {
    extern __shared__ double tw_lds[];
    tables_body(src, blockIdx.x, tw_lds);
}

// Rows of Q N (Fourier basis, Noda's kernel) in O(m) per frequency.  With
// theta = 2 pi p / m and d = j - l, a cosine row of Q gives
//   sum_{l != j} cos(theta l) / (pi (j - l))
//     = cos(theta j) (Pc(j) - Pc(m-1-j)) + sin(theta j) (Ps(j) + Ps(m-1-j)),
// Pc(t) = sum_{d=1..t} cos(theta d)/(pi d), Ps likewise with sin (the
// negative d of the sum fold onto positive ones by parity), and a sine row
//   sin(theta j) (Pc(j) - Pc(m-1-j)) - cos(theta j) (Ps(j) + Ps(m-1-j)).
// Workgroup lb handles frequency p = lb: the DC row (p = 0), the pair of
// rows 2p-1, 2p, or the Nyquist row of an even m (p = m/2); the prefix sums
// (FP64) are scanned in LDS, 16 m bytes.
template <class Src>
__device__ inline void tables_qn_body(const Src& src, int blk, double* pre) {
    __shared__ double part_c[256], part_s[256];
    int p;
    const TableJob T = src.get_q(blk, p);
    if (!(T.basis == B_FOURIER && T.hilbert == H_NODA)) return;
    const int64_t m = T.m;
    double* pc = pre;
    double* ps = pre + m;
    const int tid = threadIdx.x;
    const int64_t per = (m + 255) / 256;
    const int64_t t0 = (int64_t)tid * per, t1 = t0 + per < m ? t0 + per : m;
    double sc = 0.0, ss = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        if (t > 0) {
            double sv, cv;
            sincospi(2.0 * (double)(((int64_t)p * t) % m) / (double)m, &sv, &cv);
            const double w = 1.0 / (M_PI * (double)t);
            sc += cv * w;
            ss += sv * w;
        }
        pc[t] = sc;
        ps[t] = ss;
    }
    part_c[tid] = sc;
    part_s[tid] = ss;
    __syncthreads();
    if (tid == 0) {
        double oc = 0.0, os = 0.0;
        for (int q = 0; q < 256; ++q) {
            const double c = part_c[q], s = part_s[q];
            part_c[q] = oc;
            part_s[q] = os;
            oc += c;
            os += s;
        }
    }
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
        pc[t] += part_c[tid];
        ps[t] += part_s[tid];
    }
    __syncthreads();
    const bool nyq = (m & 1) == 0 && p == m / 2;
    for (int64_t j = tid; j < m; j += 256) {
        const double cs = pc[j] - pc[m - 1 - j], sn = ps[j] + ps[m - 1 - j];
        double sv, cv;
        sincospi(2.0 * (double)(((int64_t)p * j) % m) / (double)m, &sv, &cv);
        if (p == 0 || nyq) {
            const int64_t k = p == 0 ? 0 : m - 1;
            const double v = cv * cs + sv * sn;
            const int64_t e = (T.kp + k) * T.kt + j;
            if (T.f64) ((double*)T.table)[e] = v;
            else ((float*)T.table)[e] = (float)v;
        } else {
            const double vc = M_SQRT2 * (cv * cs + sv * sn);
            const double vs = -M_SQRT2 * (sv * cs - cv * sn);
            const int64_t e1 = (T.kp + 2 * p - 1) * T.kt + j, e2 = (T.kp + 2 * p) * T.kt + j;
            if (T.f64) {
                ((double*)T.table)[e1] = vc;
                ((double*)T.table)[e2] = vs;
            } else {
                ((float*)T.table)[e1] = (float)vc;
                ((float*)T.table)[e2] = (float)vs;
            }
        }
    }
}

template <class Src>
__global__ __launch_bounds__(256) void tables_qn_kernel(Src src) {
    extern __shared__ double pre[];
    tables_qn_body(src, blockIdx.x, pre);
}

// =========================================================================
// Centring (FP64) and per-band scales
// =========================================================================
__device__ inline double load_in(const PrepJob& J, int64_t j, int64_t col) {
    return J.in_f64 ? ((const double*)J.y)[j * J.ld + col]
                    : (double)((const float*)J.y)[j * J.ld + col];
}

// Power of two s with s * bound <= qhalf, as large as possible.
__device__ inline float pow2_scale(double qhalf, double bound) {
    if (!(bound > 0.0) || !(bound < 1e300)) return 1.0f;
    int e;
    frexp(qhalf / bound, &e);   // qhalf/bound = f 2^e, f in [0.5, 1)
    e -= 1;
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    return ldexpf(1.0f, e);
}

// Workgroup: 32 spectral points x 8 row groups.  Pass 1 sums each column
// (FP64); pass 2 subtracts the mean (FP64) and writes the centred column
// transposed (its m values contiguous) through an LDS tile.  For m <= 256
// (CACHE) the values read in pass 1 stay in registers for pass 2.  With a
// result scaling exponent alpha, a pass between them takes the column's
// sigma = sqrt(sum (y - ref)^2 / (m - 1)) (two-pass, FP64) and the centred
// column is multiplied by sigma^-alpha (1 for sigma = 0): the contraction is
// bilinear, so Phi and Psi come out divided by (sigma_1 sigma_2)^alpha.
template <class Src, bool CACHE>
__device__ inline void center_body(const PrepJob& J, int lb) {
    constexpr int CW = kCenterCols, G = 256 / kCenterCols, MAXV = 32;
    __shared__ double red[G][CW];
    __shared__ double tile[CW][64 + 1];
    const int tid = threadIdx.x, c = tid % CW, g = tid / CW;
    const int64_t col = (int64_t)lb * CW + c;
    const bool valid = col < J.n;

    double vals[CACHE ? MAXV : 1];
    if (CACHE) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k) {
            const int64_t j = g + (int64_t)G * k;
            vals[k] = (valid && j < J.m) ? load_in(J, j, col) : 0.0;
        }
    }
    double mean = 0.0;
    if (J.ref) {
        mean = valid ? J.ref[col] : 0.0;
    } else {
        double s0 = 0.0, s1 = 0.0;
        if (CACHE) {
#pragma unroll
            for (int k = 0; k < MAXV; k += 2) {
                s0 += vals[k];
                s1 += vals[k + 1];
            }
        } else if (valid) {
            int64_t j = g;
            for (; j + G < J.m; j += 2 * G) {
                s0 += load_in(J, j, col);
                s1 += load_in(J, j + G, col);
            }
            if (j < J.m) s0 += load_in(J, j, col);
        }
        red[g][c] = s0 + s1;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) t += red[q][c];
        mean = t / (double)J.m;
        __syncthreads();
    }
    if (g == 0 && valid && J.ref_out) J.ref_out[col] = mean;

    double gsc = 1.0;   // sigma^-alpha of this column
    if (J.alpha != 0.0) {
        double q0 = 0.0, q1 = 0.0;
        if (CACHE) {
#pragma unroll
            for (int k = 0; k < MAXV; k += 2) {
                const int64_t j = g + (int64_t)G * k;
                if (valid && j < J.m) q0 += (vals[k] - mean) * (vals[k] - mean);
                if (valid && j + G < J.m) q1 += (vals[k + 1] - mean) * (vals[k + 1] - mean);
            }
        } else if (valid) {
            for (int64_t j = g; j < J.m; j += G) {
                const double d = load_in(J, j, col) - mean;
                q0 += d * d;
            }
        }
        red[g][c] = q0 + q1;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) t += red[q][c];
        const double sd = sqrt(t / (double)(J.m - 1));
        if (sd > 0.0) gsc = pow(sd, -J.alpha);
        __syncthreads();
    }

    double nrm = 0.0;
    const int cc = tid / G, part = tid % G;        // writer: column cc, 8 values
    const int64_t ocol = (int64_t)lb * CW + cc;
    for (int j0 = 0; j0 < J.kt; j0 += 64) {
#pragma unroll
        for (int q = 0; q < 64 / G; ++q) {
            const int jj = g + G * q;
            const int64_t j = j0 + jj;
            double v = 0.0;
            if (valid && j < J.m) {
                if (CACHE) {
                    // j = g + G k with k = j0/G + q; j0/G is a multiple of 8
                    double x = 0.0;
#pragma unroll
                    for (int k = 0; k < MAXV; ++k)
                        if (k == j0 / G + q) x = vals[k];
                    v = (x - mean) * gsc;
                } else {
                    v = (load_in(J, j, col) - mean) * gsc;
                }
            }
            nrm += v * v;
            tile[c][jj] = v;
        }
        __syncthreads();
        const int jb = j0 + part * 8;
        if (jb < J.kt) {
            if (J.t_f64) {
                double* dst = (double*)J.yt + ocol * J.kt + jb;
#pragma unroll
                for (int e = 0; e < 8; e += 2)
                    *(double2*)(dst + e) = make_double2(tile[cc][part * 8 + e], tile[cc][part * 8 + e + 1]);
            } else {
                float* dst = (float*)J.yt + ocol * J.kt + jb;
#pragma unroll
                for (int e = 0; e < 8; e += 4)
                    *(float4*)(dst + e) = make_float4((float)tile[cc][part * 8 + e], (float)tile[cc][part * 8 + e + 1],
                                                      (float)tile[cc][part * 8 + e + 2], (float)tile[cc][part * 8 + e + 3]);
            }
        }
        __syncthreads();
    }
    red[g][c] = nrm;
    __syncthreads();
    if (g == 0) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) tot += red[q][c];
        const double r = sqrt(tot);
        float sa = 1.0f, sb = 1.0f;
        if (J.scale) {
            sa = pow2_scale(J.qhalf, J.boundA * r);
            sb = pow2_scale(J.qhalf, J.boundB * r);
        }
        if (J.sA) J.sA[col] = sa;
        if (J.sB) J.sB[col] = sb;
    }
}

template <class Src>
__device__ inline void center_dispatch(const Src& src, int blk) {
    int lb;
    const PrepJob J = src.get(blk, lb);
    if (J.m <= 256) center_body<Src, true>(J, lb);
    else center_body<Src, false>(J, lb);
}

template <class Src>
__global__ __launch_bounds__(256) void center_kernel(Src src) {
    center_dispatch(src, blockIdx.x);
}

// The three preparation kernels of a single or heterocorrelation call on the
// table-product path in one launch (they are independent of each other):
// workgroups [0, nt) build the table, [nt, nt + nq) its Q N rows, the rest
// centre the spectra.  Dynamic LDS: 32 m bytes (the table kernel's; the
// Q N rows use the first 16 m).  Saves two launches per call, which is
// what a small problem costs.
__global__ __launch_bounds__(256) void prep_kernel(TableSrcInline ts, int nt, int nq, PrepSrcInline ps) {
    extern __shared__ double prep_lds[];
    const int b = blockIdx.x;
    if (b < nt) tables_body(ts, b, prep_lds);
    else if (b < nt + nq) tables_qn_body(ts, b - nt, prep_lds);
    else center_dispatch(ps, b - nt - nq);
}

// =========================================================================
// Transform GEMM: [A | B] = Yc^T T^T, then scale, round and pack
// =========================================================================
// Four consecutive contraction elements (k .. k+3 of one row, idx a multiple
// of 4, so one vector store per plane) rounded to the operand format: split
// BF16 stores hi = RNE(x) and lo = RNE(x - hi).
template <int P>
__device__ inline void store_operand4(void* p0, void* p1, int64_t idx, const float (&x)[4]) {
    if constexpr (P == P_F32) {
        *(float4*)((float*)p0 + idx) = make_float4(x[0], x[1], x[2], x[3]);
    } else if constexpr (P == P_SPLIT || P == P_BF16) {
        uint32_t hw[2], lw[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) bf16x2_split(x[2 * q], x[2 * q + 1], hw[q], lw[q]);
        *(uint2*)((uint16_t*)p0 + idx) = make_uint2(hw[0], hw[1]);
        if constexpr (P == P_SPLIT) *(uint2*)((uint16_t*)p1 + idx) = make_uint2(lw[0], lw[1]);
    } else if constexpr (P == P_F16) {
        *(h4v*)((_Float16*)p0 + idx) = h4v{(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
    } else if constexpr (P == P_SPLIT16) {
        h4v hi, lo;
        f16x4_split(x, hi, lo);
        *(h4v*)((_Float16*)p0 + idx) = hi;
        *(h4v*)((_Float16*)p1 + idx) = lo;
    } else if constexpr (P == P_FP8) {
        *(uint32_t*)((uint8_t*)p0 + idx) = fp8_e4m3_rne(x[0]) | ((uint32_t)fp8_e4m3_rne(x[1]) << 8) |
                                           ((uint32_t)fp8_e4m3_rne(x[2]) << 16) | ((uint32_t)fp8_e4m3_rne(x[3]) << 24);
    }
}

// FP64 transform GEMM (the FP64 contraction's operands, no rounding to a
// narrower format): 64 x 64 workgroup tiles, each wave 32 x 32 (2 x 2 blocks
// of v_mfma_f64_16x16x4f64).
template <int P, class Src>
__global__ __launch_bounds__(256) void transform_kernel(Src src) {
    static_assert(P == P_F64, "the reduced precisions use transform32_kernel");
    int lb;
    const PrepJob J = src.get(blockIdx.x, lb);
    const int row_tiles = J.rows_pad / kTransformTile;
    const int bi = lb / row_tiles, br = lb % row_tiles;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = (int64_t)bi * kTransformTile + (wave >> 1) * 32;
    const int64_t r0 = (int64_t)br * kTransformTile + (wave & 1) * 32;
    if (r0 >= J.rows_pad) return;

    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
    const double* Y = (const double*)J.yt;
    const double* T = (const double*)J.table;
    for (int k0 = 0; k0 < J.kt; k0 += 16) {
        d4 fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fa[a] = *(const d4*)(Y + (i0 + a * 16 + row16) * J.kt + k0 + kg * 4);
#pragma unroll
        for (int b = 0; b < 2; ++b) fb[b] = *(const d4*)(T + (r0 + b * 16 + row16) * J.kt + k0 + kg * 4);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a][s], fb[b][s], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t r = r0 + b * 16 + row16;
            if (r >= 2 * (int64_t)J.kp) continue;
            const bool isB = r >= J.kp;
            if (isB && !J.need_b) continue;
            const int64_t k = isB ? r - J.kp : r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = i0 + a * 16 + kg + 4 * q;   // FP64 accumulator rows
                double* dst = (double*)(isB ? J.B0 : J.A0);
                dst[i * J.kp + k] = acc[a][b][q];
            }
        }
}

// FP32 transform GEMM for the reduced precisions.  Workgroup tile: 64
// spectral points x 256 transform rows; each wave owns 64 x 64 (4 x 4 blocks
// of v_mfma_f32_16x16x4f32) and prefetches the next K step's fragments while
// the current step's MFMAs run.  The table rows are the MFMA's A operand, so
// accumulator register q of lane l holds transform row 4(l/16) + q of point
// l%16: four consecutive contraction elements of one operand row, which the
// epilogue stores with one vector store per plane (16 lanes cover a
// contiguous run of the blocked layout).
constexpr int kT32Cols = 256;

template <int P, class Src>
__global__ __launch_bounds__(256) void transform32_kernel(Src src) {
    int lb;
    const PrepJob J = src.get(blockIdx.x, lb);
    const int rtiles = (J.rows_pad + kT32Cols - 1) / kT32Cols;
    const int bi = lb / rtiles, br = lb % rtiles;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = (int64_t)bi * 64;
    const int64_t r0 = (int64_t)br * kT32Cols + wave * 64;
    // The per-band scales of the workgroup's 64 spectral points (A then B),
    // read once ahead of the K loop and kept in LDS: read between the
    // epilogue's stores, each load's wait would also wait for every store
    // before it (vmcnt counts both).
    // A set whose B operand is not needed (the left set of a
    // heterocorrelation) has no B scales: sB is null then.
    __shared__ float s_scale[2][64];
    const int st = threadIdx.x;
    const float* sp = st < 64 ? J.sA : J.sB;
    const float scv = (st < 128 && sp != nullptr) ? sp[i0 + (st & 63)] : 0.0f;
    // waves past the transform's rows skip the work but still take the barrier
    const bool active = r0 < J.rows_pad;
    const float* Y = (const float*)J.yt;
    const float* T = (const float*)J.table;
    const float* yrow[4];
    const float* trow[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        yrow[a] = Y + (i0 + a * 16 + row16) * J.kt + kg * 4;
        trow[a] = T + (r0 + a * 16 + row16) * J.kt + kg * 4;
    }
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
    f4 fa[4], fb[4];
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            fa[a] = *(const f4*)(yrow[a]);
            fb[a] = *(const f4*)(trow[a]);
        }
    }
    for (int k0 = 0; active && k0 < J.kt; k0 += 16) {
        f4 na[4], nb[4];
        const bool more = k0 + 16 < J.kt;
        if (more) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                na[a] = *(const f4*)(yrow[a] + k0 + 16);
                nb[a] = *(const f4*)(trow[a] + k0 + 16);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[b][s], fa[a][s], acc[a][b], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                fa[a] = na[a];
                fb[a] = nb[a];
            }
        }
    }
    if (st < 128) s_scale[st >> 6][st & 63] = scv;
    __syncthreads();
    if (!active) return;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        // rows r0 + 16 b .. + 15 are all A rows or all B rows (K is a
        // multiple of 16); this lane holds rows rb .. rb + 3
        const int64_t rb0 = r0 + b * 16;
        if (rb0 >= 2 * (int64_t)J.kp) continue;
        const bool isB = rb0 >= J.kp;
        if (isB && !J.need_b) continue;
        const int64_t k = (isB ? rb0 - J.kp : rb0) + kg * 4;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int il = a * 16 + row16;
            const int64_t i = i0 + il;
            const float sc = s_scale[isB ? 1 : 0][il];
            const float x[4] = {acc[a][b][0] * sc, acc[a][b][1] * sc, acc[a][b][2] * sc, acc[a][b][3] * sc};
            const int64_t idx = blocked_layout(P) ? blocked_index(i, k, J.kp) : i * J.kp + k;
            store_operand4<P>(isB ? J.B0 : J.A0, isB ? J.B1 : J.A1, idx, x);
        }
    }
}

// Centring fused into the FP32 transform GEMM, for short spectra (kt <=
// kFusedTransformMaxK): each workgroup centres its own 64 spectral points
// (the mean over the m perturbation steps in FP64, or the given reference,
// Sec. 2 Eqs. (dynspec), (ref)), applies the result scaling sigma^-alpha,
// takes each column's norm for the per-band scales, and keeps the centred
// columns in LDS as the GEMM's B operand, so the centred spectra never go
// through HBM.  The arithmetic per value is the
// separate centring kernel's (FP64 difference and scaling, one rounding to
// FP32); only the order of the FP64 column sums differs.  One workgroup per
// 64 spectral points: it centres them once and then runs every row tile of
// 256 transform rows over them in turn (m up to 128 has one, up to 256 two).
template <int P, class Src>
__global__ __launch_bounds__(256) void center_transform32_kernel(Src src) {
    constexpr int YP = kFusedTransformMaxK + 4;   // LDS row pitch of a centred column (floats)
    __shared__ __attribute__((aligned(16))) float ytile[64 * YP];
    __shared__ double red[4][64];
    __shared__ float s_scale[2][64];
    int lb;
    const PrepJob J = src.get(blockIdx.x, lb);
    const int rtiles = (J.rows_pad + kT32Cols - 1) / kT32Cols;
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)lb * 64;

    // centring: thread (g, c) takes rows g, g + 4, ... of column i0 + c, all
    // loaded at once into registers (the LDS tile already limits the kernel
    // to two workgroups per CU, so the registers are free)
    {
        constexpr int NV = kFusedTransformMaxK / 4;
        const int c = tid & 63, g = tid >> 6;
        const int64_t col = i0 + c;
        const bool valid = col < J.n;
        double vals[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int j = g + 4 * k;
            vals[k] = (valid && j < J.m) ? load_in(J, j, col) : 0.0;
        }
        double mean = 0.0;
        if (J.ref) {
            mean = valid ? J.ref[col] : 0.0;
        } else {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < NV; k += 2) {
                s0 += vals[k];
                s1 += vals[k + 1];
            }
            red[g][c] = s0 + s1;
            __syncthreads();
            mean = (red[0][c] + red[1][c] + red[2][c] + red[3][c]) / (double)J.m;
            __syncthreads();
        }
        double gsc = 1.0;
        if (J.alpha != 0.0) {
            double q0 = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const double d = vals[k] - mean;
                if (valid && g + 4 * k < J.m) q0 += d * d;
            }
            red[g][c] = q0;
            __syncthreads();
            const double sd = sqrt((red[0][c] + red[1][c] + red[2][c] + red[3][c]) / (double)(J.m - 1));
            if (sd > 0.0) gsc = pow(sd, -J.alpha);
            __syncthreads();
        }
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int j = g + 4 * k;
            const double v = (valid && j < J.m) ? (vals[k] - mean) * gsc : 0.0;
            nrm += v * v;
            if (j < J.kt) ytile[c * YP + j] = (float)v;
        }
        red[g][c] = nrm;
        __syncthreads();
        if (g == 0) {
            const double r = sqrt(red[0][c] + red[1][c] + red[2][c] + red[3][c]);
            float sa = 1.0f, sb = 1.0f;
            if (J.scale) {
                sa = pow2_scale(J.qhalf, J.boundA * r);
                sb = pow2_scale(J.qhalf, J.boundB * r);
            }
            s_scale[0][c] = J.sA ? sa : 0.0f;
            s_scale[1][c] = J.sB ? sb : 0.0f;
            if (valid && J.ref_out) J.ref_out[col] = mean;
            if (J.sA) J.sA[col] = sa;
            if (J.sB) J.sB[col] = sb;
        }
        __syncthreads();
    }

    const int lane = tid & 63, wave = tid >> 6;
    const int row16 = lane & 15, kg = lane >> 4;
    const float* T = (const float*)J.table;
    // no barrier below: the LDS tile and the scales are only read from here on
    for (int br = 0; br < rtiles; ++br) {
        const int64_t r0 = (int64_t)br * kT32Cols + wave * 64;
        if (r0 >= J.rows_pad) break;
        const float* yrow[4];
        const float* trow[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            yrow[a] = ytile + (a * 16 + row16) * YP + kg * 4;
            trow[a] = T + (r0 + a * 16 + row16) * J.kt + kg * 4;
        }
        f4 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
        for (int k0 = 0; k0 < J.kt; k0 += 16) {
            f4 fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                fa[a] = *(const f4*)(yrow[a] + k0);
                fb[a] = *(const f4*)(trow[a] + k0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[b][s], fa[a][s], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t rb0 = r0 + b * 16;
            if (rb0 >= 2 * (int64_t)J.kp) continue;
            const bool isB = rb0 >= J.kp;
            if (isB && !J.need_b) continue;
            const int64_t k = (isB ? rb0 - J.kp : rb0) + kg * 4;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int il = a * 16 + row16;
                const int64_t i = i0 + il;
                const float sc = s_scale[isB ? 1 : 0][il];
                const float x[4] = {acc[a][b][0] * sc, acc[a][b][1] * sc, acc[a][b][2] * sc, acc[a][b][3] * sc};
                const int64_t idx = blocked_layout(P) ? blocked_index(i, k, J.kp) : i * J.kp + k;
                store_operand4<P>(isB ? J.B0 : J.A0, isB ? J.B1 : J.A1, idx, x);
            }
        }
    }
}

// =========================================================================
// Radix FFT transform (power-of-two m)
// =========================================================================
// For m = 2^s, 128 <= m <= 1024, the perturbation-axis transform runs as
// FFTs of length L = 2m in LDS instead of the product with the table (m^2
// work per spectral point becomes m log m), in FP64 for the FP64 path and
// FP32 otherwise.  Two spectral points y1, y2
// travel as one complex sequence z = y1 + i y2, zero padded to L:
//   Z = FFT_L(z).  Its even bins are the m-point spectra of the pair,
//       Y1(p) = (Z(2p) + conj Z(L-2p)) / 2 and Y2(p) = (Z(2p) - conj Z(L-2p)) / 2i
//       (Eq. (disFT)), packed into A's rows as the table's rows pack them.
//   Noda's kernel (Eq. (HilbNoda)): (N y)_j = sum_d h(d) y_(j+d) with
//       h(d) = 1/(pi d), d != 0, is a linear correlation; the zero padding
//       makes the circular correlation of length L equal to it on j < m, so
//       r = N z = IFFT_L(Z . i G) with G(w) = (2/L) sum_{d=1}^{m-1} h(d)
//       sin(2 pi w d / L) (the DFT of h is -2i sum h(d) sin(...)).  B's rows
//       are the packed m-point spectra of r1 + i r2 = r, taken as the even
//       bins of the FFT_L of r with its entries from m on set to zero.  The
//       inverse runs as a forward FFT between conjugations.
//   Circular kernel (and the R code's bin list): B's rows are those of
//       i Y (each (Re, Im) pair becomes (-Im, Re)), DC and Nyquist zero.
//   Time basis (Noda's kernel): A is the centred spectrum itself and B is r.
// Each pair is transformed by G = L/8 threads holding 8 values each; a pass
// of radix R (8, then 4 or 2 for the last) is a Stockham step in place of
// the usual bit reversal, so every FFT leaves its output in natural order.
// Two LDS buffers per pair alternate between passes (one barrier per pass).
// LDS indices are padded by one entry in 16 against bank conflicts.  The
// twiddles of each pass and the Noda multiplier depend only on the thread's
// index within its pair, so each thread keeps its own in registers.
// Complex values are float2 (reduced formats) or double2 (FP64 path).
template <class V> struct Scal;
template <> struct Scal<float2> { using T = float; };
template <> struct Scal<double2> { using T = double; };
__device__ inline float2 cx(float a, float b) { return make_float2(a, b); }
__device__ inline double2 cx(double a, double b) { return make_double2(a, b); }
template <class V> __device__ inline V cadd(V a, V b) { return cx(a.x + b.x, a.y + b.y); }
template <class V> __device__ inline V csub(V a, V b) { return cx(a.x - b.x, a.y - b.y); }
template <class V> __device__ inline V cmul(V a, V b) {
    return cx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class V> __device__ inline V mul_mi(V a) { return cx(a.y, -a.x); }   // a * (-i)
__device__ inline int fpad(int i) { return i + (i >> 4); }

// In-register forward DFTs (exp(-2 pi i j k / R)) of v[O .. O+R-1], outputs
// in natural order.
template <int O, class V>
__device__ inline void dft2(V (&v)[8]) {
    const V a = v[O];
    v[O] = cadd(a, v[O + 1]);
    v[O + 1] = csub(a, v[O + 1]);
}
template <int O, int S = 1, class V>
__device__ inline void dft4(V (&v)[8]) {
    const V a0 = cadd(v[O], v[O + 2 * S]), a1 = csub(v[O], v[O + 2 * S]);
    const V a2 = cadd(v[O + S], v[O + 3 * S]), a3 = mul_mi(csub(v[O + S], v[O + 3 * S]));
    v[O] = cadd(a0, a2);
    v[O + 2 * S] = csub(a0, a2);
    v[O + S] = cadd(a1, a3);
    v[O + 3 * S] = csub(a1, a3);
}
template <class V>
__device__ inline void dft8(V (&v)[8]) {
    using S = typename Scal<V>::T;
    constexpr S r = S(0.70710678118654752440);
    // E = DFT4 of the even inputs, O = DFT4 of the odd ones (in place, stride 2)
    dft4<0, 2>(v);
    dft4<1, 2>(v);
    // X_k = E_k + W^k O_k, X_(k+4) = E_k - W^k O_k, W = exp(-i pi / 4)
    const V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    const V o0 = v[1];
    const V o1 = cx(r * (v[3].x + v[3].y), r * (v[3].y - v[3].x));
    const V o2 = mul_mi(v[5]);
    const V o3 = cx(r * (v[7].y - v[7].x), -r * (v[7].x + v[7].y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// dft8 of inputs whose last four are zero (the zero-padded half of a
// first pass).
template <class V>
__device__ inline void dft8_half(V (&v)[8]) {
    using S = typename Scal<V>::T;
    constexpr S r = S(0.70710678118654752440);
    const V e0 = cadd(v[0], v[2]), e2 = csub(v[0], v[2]);
    const V e1 = cadd(v[0], mul_mi(v[2])), e3 = csub(v[0], mul_mi(v[2]));
    const V q0 = cadd(v[1], v[3]), q2 = csub(v[1], v[3]);
    const V q1 = cadd(v[1], mul_mi(v[3])), q3 = csub(v[1], mul_mi(v[3]));
    const V o1 = cx(r * (q1.x + q1.y), r * (q1.y - q1.x));
    const V o2 = mul_mi(q2);
    const V o3 = cx(r * (q3.y - q3.x), -r * (q3.x + q3.y));
    v[0] = cadd(e0, q0);
    v[4] = csub(e0, q0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <int L> struct FftCfg {
    static constexpr int G = L / 8;              // threads per pair
    static constexpr int PW = 256 / G;           // pairs per pass of the workgroup
    static constexpr int BUF = L + L / 16;       // padded entries of one buffer
    static constexpr int PAIR = 2 * BUF + 4;     // LDS entries per pair (staggered banks)
    static constexpr int PTS = fft_points(L);    // spectral points per workgroup
    static constexpr int ITER = PTS / (2 * PW);
    static constexpr int NPASS = (__builtin_ctz(L) + 2) / 3;
    static constexpr int RG = 256 / PTS;         // row groups of the fused centring
    static constexpr int MV = (L / 2) / RG;      // centred values per thread
    static constexpr int ZS = L / 2 + 4;         // scalar stride of a staged column
    static_assert(ITER >= 1 && PTS % (2 * PW) == 0, "workgroup shape");
    static_assert(RG * MV == L / 2 && MV % 2 == 0, "centring shape");
};

// Centring of the workgroup's PTS spectral points, fused ahead of the FFTs
// (Eqs. (dynspec), (ref); the arithmetic of center_body): thread
// (c, g) = (tid % PTS, tid / PTS) reads rows g + RG k of column p0 + c,
// m = L/2 rows in all.  The column mean (or the caller's reference) and,
// with a result scaling exponent alpha, sigma^-alpha are FP64 sums reduced
// through LDS; the column norm gives the per-band scales, which go to the
// job's scale vectors (the contraction reads them there).  The centred
// values enter the FFTs divided by a power of two 2^e near the column norm
// (exact), and s_sc carries the operand scale times 2^e, which the emitted
// rows are multiplied by: the two columns that share a complex FFT then
// enter at unit norm, so the rounding-level cross-talk of their separation
// stays relative to each column's own norm (a weak spectral variable next
// to a strong one keeps its accuracy).  The values stay in registers (as
// float for the reduced formats).
template <int L, class S>
__device__ inline void fft_center(const PrepJob& J, int64_t p0, int tid, S (&xf)[FftCfg<L>::MV],
                                  S* s_sc, double* red) {
    constexpr int PTS = FftCfg<L>::PTS, RG = FftCfg<L>::RG, MV = FftCfg<L>::MV;
    const int c = tid % PTS, g = tid / PTS;
    const int64_t col = p0 + c;
    const bool valid = col < J.n;
    double v[MV];
#pragma unroll
    for (int k = 0; k < MV; ++k) v[k] = valid ? load_in(J, g + (int64_t)RG * k, col) : 0.0;
    auto colsum = [&](double x) {
        red[g * PTS + c] = x;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < RG; ++q) t += red[q * PTS + c];
        __syncthreads();
        return t;
    };
    double mean;
    if (J.ref) {
        mean = valid ? J.ref[col] : 0.0;
    } else {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < MV; k += 2) {
            s0 += v[k];
            s1 += v[k + 1];
        }
        mean = colsum(s0 + s1) / (double)J.m;
    }
    double gsc = 1.0;   // sigma^-alpha of this column
    if (J.alpha != 0.0) {
        double q0 = 0.0;
#pragma unroll
        for (int k = 0; k < MV; ++k) q0 += (v[k] - mean) * (v[k] - mean);
        const double sd = sqrt(colsum(valid ? q0 : 0.0) / (double)(J.m - 1));
        if (sd > 0.0) gsc = pow(sd, -J.alpha);
    }
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        const double x = valid ? (v[k] - mean) * gsc : 0.0;
        nrm += x * x;
    }
    const double r = sqrt(colsum(nrm));
    int e = 0;
    if (r > 0.0) frexp(r, &e);   // r = f 2^e, f in [0.5, 1)
    e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
    const double down = ldexp(1.0, -e);
#pragma unroll
    for (int k = 0; k < MV; ++k) xf[k] = (S)((valid ? (v[k] - mean) * gsc : 0.0) * down);
    if (g == 0) {
        float sa = 1.0f, sb = 1.0f;
        if (J.scale) {
            sa = pow2_scale(J.qhalf, J.boundA * r);
            sb = pow2_scale(J.qhalf, J.boundB * r);
        }
        s_sc[c] = (S)ldexp((double)sa, e);
        s_sc[PTS + c] = (S)ldexp((double)sb, e);
        if (J.sA) J.sA[col] = sa;
        if (J.sB) J.sB[col] = sb;
        if (valid && J.ref_out) J.ref_out[col] = mean;
    }
}

// This thread's twiddles: pass q (stride NS, radix R) multiplies input r of
// its butterfly b by exp(-2 pi i r k / (NS R)), k = (t + b G) mod NS.
template <int L, class V> struct FftTw { V w[FftCfg<L>::NPASS][8]; };

template <int L, class V, int NS = 1, int PASS = 0>
__device__ inline void fft_twiddles(FftTw<L, V>& tw, const V* tab, int t) {
    constexpr int R = (L / NS) >= 8 ? 8 : L / NS, NB = 8 / R, STEP = L / (NS * R);
    if constexpr (NS > 1) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 1; r < R; ++r) tw.w[PASS][b * R + r] = tab[r * ((t + b * FftCfg<L>::G) & (NS - 1)) * STEP];
    }
    if constexpr (NS * R < L) fft_twiddles<L, V, NS * R, PASS + 1>(tw, tab, t);
}

// One Stockham pass of radix R at stride NS: butterfly j (this thread's
// j = t + b G, b < 8/R) takes inputs j + r L/R (held in v), applies the
// twiddles exp(-2 pi i r (j mod NS) / (NS R)), transforms, and writes output
// r to (j div NS) NS R + (j mod NS) + r NS.
template <int L, int R, int NS, bool HALF, class V>
__device__ inline void fft_pass(V (&v)[8], V* dst, const V (&tw)[8], int t) {
    constexpr int G = L / 8, NB = 8 / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * G, k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], tw[b * R + r]);
        }
        if constexpr (R == 8 && HALF) dft8_half(v);
        else if constexpr (R == 8) dft8(v);
        else if constexpr (R == 4) { if (b == 0) dft4<0>(v); else dft4<4>(v); }
        else {
            if (b == 0) dft2<0>(v);
            else if (b == 1) dft2<2>(v);
            else if (b == 2) dft2<4>(v);
            else dft2<6>(v);
        }
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[fpad(base + r * NS)] = v[b * R + r];
    }
}

template <int L, int R, class V>
__device__ inline void fft_load(V (&v)[8], const V* src, int t) {
    constexpr int G = L / 8, NB = 8 / R;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = src[fpad(t + b * G + r * (L / R))];
}

// Forward FFT of the pair whose first-pass inputs v[r] = z(t + r G) this
// thread holds (HALF: v[4..7] are zero).  Passes write base + off and
// base + (off ^ BUF) in turn; returns the offset of the buffer holding the
// natural-order output (after a workgroup barrier).
template <int L, bool HALF, class V, int NS = 1, int PASS = 0>
__device__ inline int fft_run(V (&v)[8], V* base, int off, const FftTw<L, V>& tw, int t) {
    constexpr int R = (L / NS) >= 8 ? 8 : L / NS;
    fft_pass<L, R, NS, HALF && NS == 1>(v, base + off, tw.w[PASS], t);
    __syncthreads();
    if constexpr (NS * R < L) {
        constexpr int R2 = (L / (NS * R)) >= 8 ? 8 : L / (NS * R);
        fft_load<L, R2>(v, base + off, t);
        return fft_run<L, HALF, V, NS * R, PASS + 1>(v, base, off ^ FftCfg<L>::BUF, tw, t);
    } else {
        return off;
    }
}

// Rows k0 .. k0+7 (k0 a multiple of 8) of the packed half spectrum of one
// point of a pair, from the pair's natural-order L-point spectrum Z: row 0
// is Re Y(0), rows 2p-1, 2p are sqrt2 Re Y(p), sqrt2 Im Y(p), row m-1 is
// Re Y(m/2).  rot: rows of i Y with DC and Nyquist zero; zero_nyq: the
// Nyquist row is zero.
template <int L, class V, class S>
__device__ inline void packed_rows8(const V* Z, bool second, int k0, bool rot, bool zero_nyq, S (&x)[8]) {
    constexpr int M = L / 2;
    constexpr S hf = S(0.5), s2 = S(0.70710678118654752440);
    S yr[5], yi[5];   // 2 Re Y(p), 2 Im Y(p) for p = k0/2 .. k0/2 + 4
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int p = (k0 >> 1) + q;
        const V a = Z[fpad(2 * p)], b = Z[fpad((L - 2 * p) & (L - 1))];
        yr[q] = second ? a.y + b.y : a.x + b.x;
        yi[q] = second ? b.x - a.x : a.y - b.y;
    }
    if (!rot) {
        x[0] = k0 == 0 ? hf * yr[0] : s2 * yi[0];
        x[1] = s2 * yr[1];
        x[2] = s2 * yi[1];
        x[3] = s2 * yr[2];
        x[4] = s2 * yi[2];
        x[5] = s2 * yr[3];
        x[6] = s2 * yi[3];
        x[7] = k0 + 7 == M - 1 ? (zero_nyq ? S(0) : hf * yr[4]) : s2 * yr[4];
    } else {
        x[0] = k0 == 0 ? S(0) : s2 * yr[0];
        x[1] = -s2 * yi[1];
        x[2] = s2 * yr[1];
        x[3] = -s2 * yi[2];
        x[4] = s2 * yr[2];
        x[5] = -s2 * yi[3];
        x[6] = s2 * yr[3];
        x[7] = k0 + 7 == M - 1 ? S(0) : -s2 * yi[4];
    }
}

// Eight consecutive contraction elements of one operand row (idx a multiple
// of 8) rounded to the operand format, one vector store per plane (FP64:
// stored as they are).
template <int P, class S>
__device__ inline void store_operand8(void* p0, void* p1, int64_t idx, const S (&x)[8]) {
    if constexpr (P == P_F64) {
        double2* d = (double2*)((double*)p0 + idx);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = make_double2(x[2 * q], x[2 * q + 1]);
    } else if constexpr (P == P_F32) {
        float4* d = (float4*)((float*)p0 + idx);
        d[0] = make_float4(x[0], x[1], x[2], x[3]);
        d[1] = make_float4(x[4], x[5], x[6], x[7]);
    } else if constexpr (P == P_SPLIT || P == P_BF16) {
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bf16x2_split(x[2 * q], x[2 * q + 1], hw[q], lw[q]);
        *(uint4*)((uint16_t*)p0 + idx) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        if constexpr (P == P_SPLIT) *(uint4*)((uint16_t*)p1 + idx) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    } else if constexpr (P == P_F16) {
        *(h8*)((_Float16*)p0 + idx) = h8{(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3],
                                         (_Float16)x[4], (_Float16)x[5], (_Float16)x[6], (_Float16)x[7]};
    } else if constexpr (P == P_SPLIT16) {
        h4v h0, l0, h1, l1;
        f16x4_split(x, h0, l0);
        f16x4_split(x + 4, h1, l1);
        *(h8*)((_Float16*)p0 + idx) = h8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
        *(h8*)((_Float16*)p1 + idx) = h8{l0[0], l0[1], l0[2], l0[3], l1[0], l1[1], l1[2], l1[3]};
    } else if constexpr (P == P_FP8) {
        uint32_t w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
            w[q] = fp8_e4m3_rne(x[4 * q]) | ((uint32_t)fp8_e4m3_rne(x[4 * q + 1]) << 8) |
                   ((uint32_t)fp8_e4m3_rne(x[4 * q + 2]) << 16) | ((uint32_t)fp8_e4m3_rne(x[4 * q + 3]) << 24);
        *(uint2*)((uint8_t*)p0 + idx) = make_uint2(w[0], w[1]);
    }
}

// One operand's rows for the 2 PW points of a pass: 256 tasks of 8 rows.
// Blocked layout: lanes in pairs cover the two halves of one point's K
// block, consecutive pairs consecutive points (one contiguous run per
// block); row layout: consecutive lanes cover consecutive rows of a point.
// seq (time basis): the rows are the sequence itself -- A the centred
// spectrum staged in the pair's buffer, B the correlation r = conj(U) held
// there.
template <int P> using FftV = typename std::conditional<P == P_F64, double2, float2>::type;
template <int P> using FftS = typename std::conditional<P == P_F64, double, float>::type;

template <int P, int L>
__device__ inline void fft_emit(const PrepJob& J, int64_t i0, const FftV<P>* bufs, int off, int tid,
                                bool isB, bool rot, bool zero_nyq, bool seq, const FftS<P>* s_sc, int pt0) {
    using V = FftV<P>;
    using S = FftS<P>;
    constexpr int M = L / 2, NP = 2 * FftCfg<L>::PW;
    int pt, hb;
    if constexpr (blocked_layout(P)) {
        const int u = tid >> 1;
        pt = u % NP;
        hb = 2 * (u / NP) + (tid & 1);
    } else {
        pt = tid / (M / 8);
        hb = tid % (M / 8);
    }
    const V* Z = bufs + (pt >> 1) * FftCfg<L>::PAIR + off;
    S x[8];
    if (!seq) {
        packed_rows8<L>(Z, pt & 1, 8 * hb, rot, zero_nyq, x);
    } else if (isB) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const V u = Z[fpad(8 * hb + e)];
            x[e] = (pt & 1) ? -u.y : u.x;
        }
    } else {
        const S* src = (const S*)Z + (pt & 1) * FftCfg<L>::ZS + 8 * hb;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = src[e];
    }
    const S sc = s_sc[(isB ? FftCfg<L>::PTS : 0) + pt0 + pt];
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] *= sc;
    const int64_t i = i0 + pt, k = 8 * hb;
    const int64_t idx = blocked_layout(P) ? blocked_index(i, k, J.kp) : i * J.kp + k;
    store_operand8<P>(isB ? J.B0 : J.A0, isB ? J.B1 : J.A1, idx, x);
}

template <int P, int LOG2L, class Src>
__global__ __launch_bounds__(256) void fft_transform_kernel(Src src) {
    constexpr int L = 1 << LOG2L;
    using C = FftCfg<L>;
    using V = FftV<P>;
    using S = FftS<P>;
    __shared__ V s_buf[C::PW * C::PAIR];
    __shared__ S s_sc[2 * C::PTS];
    __shared__ double s_red[256];
    int lb;
    const PrepJob J = src.get(blockIdx.x, lb);
    const int tid = threadIdx.x, grp = tid / C::G, t = tid % C::G;
    const bool noda = J.need_b && J.hilbert == H_NODA;
    const bool rcompat = J.hilbert == H_R_COMPAT;
    const bool tbasis = J.basis == B_TIME;   // (Noda's kernel only)
    const int64_t p0 = (int64_t)lb * C::PTS;   // first spectral point of the workgroup
    const V* tab = (const V*)J.table;
    FftTw<L, V> tw;
    fft_twiddles<L>(tw, tab, t);
    S gr[8];   // Noda multiplier G(t + r G)
#pragma unroll
    for (int r = 0; r < 8; ++r) gr[r] = noda ? ((const S*)(tab + L))[t + r * C::G] : S(0);
    S xf[C::MV];
    fft_center<L>(J, p0, tid, xf, s_sc, s_red);
    V* mine = s_buf + grp * C::PAIR;
    int off = 0;   // buffer holding the last FFT output (all pairs alike)
#pragma unroll 1
    for (int it = 0; it < C::ITER; ++it) {
        const int pt0 = it * 2 * C::PW;
        const int64_t i0 = p0 + pt0;
        // stage the pass's 2 PW centred columns in buffer `off`, which the
        // first FFT pass leaves alone (its second pass overwrites it, after
        // a barrier that every read of the staged values precedes)
        __syncthreads();   // the previous pass's readers of buffer `off` are done
        {
            const int lc = tid % C::PTS - pt0, g = tid / C::PTS;
            if (lc >= 0 && lc < 2 * C::PW) {
                S* zt = (S*)(s_buf + (lc >> 1) * C::PAIR + off) + (lc & 1) * C::ZS;
#pragma unroll
                for (int k = 0; k < C::MV; ++k) zt[g + C::RG * k] = xf[k];
            }
        }
        __syncthreads();
        const S* y1 = (const S*)(mine + off);
        V v[8];
        if (tbasis) fft_emit<P, L>(J, i0, s_buf, off, tid, false, false, false, true, s_sc, pt0);
        if (!tbasis || noda) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = cx(y1[t + r * C::G], y1[C::ZS + t + r * C::G]);
#pragma unroll
            for (int r = 4; r < 8; ++r) v[r] = cx(S(0), S(0));
            off = fft_run<L, true>(v, mine, off ^ C::BUF, tw, t);
        }
        if (!tbasis) fft_emit<P, L>(J, i0, s_buf, off, tid, false, false, rcompat, false, s_sc, pt0);
        if (J.need_b && !noda) fft_emit<P, L>(J, i0, s_buf, off, tid, true, true, false, false, s_sc, pt0);
        if (noda) {
            // conj(i G Z): the inverse transform as a forward one
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const V z = mine[off + fpad(t + r * C::G)];
                v[r] = cx(-gr[r] * z.y, -gr[r] * z.x);
            }
            off = fft_run<L, false>(v, mine, off ^ C::BUF, tw, t);
            if (tbasis) {
                fft_emit<P, L>(J, i0, s_buf, off, tid, true, false, false, true, s_sc, pt0);
            } else {
                // r = conj of that, entries from m on dropped
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const V u = mine[off + fpad(t + r * C::G)];
                    v[r] = cx(u.x, -u.y);
                }
#pragma unroll
                for (int r = 4; r < 8; ++r) v[r] = cx(S(0), S(0));
                off = fft_run<L, true>(v, mine, off ^ C::BUF, tw, t);
                fft_emit<P, L>(J, i0, s_buf, off, tid, true, false, false, false, s_sc, pt0);
            }
        }
    }
}

// Tables of the radix FFT transform, L = 2m: tw[w] = exp(-2 pi i w / L) and,
// for Noda's kernel, g[w] = (2/L) sum_{d=1}^{m-1} sin(2 pi w d / L) / (pi d)
// (FP64 sums, stored as double for the FP64 path, else as float; g follows
// the L twiddles).  One workgroup per w.
template <class Src>
__global__ __launch_bounds__(256) void fft_tables_kernel(Src src) {
    __shared__ double part[256];
    int w;
    const TableJob T = src.get_q(blockIdx.x, w);
    const int64_t m = T.m, L = 2 * m;
    const int tid = threadIdx.x;
    double s = 0.0;
    if (T.hilbert == H_NODA) {
        for (int64_t d = tid + 1; d < m; d += 256) {
            double sv, cv;
            sincospi(2.0 * (double)(((int64_t)w * d) % L) / (double)L, &sv, &cv);
            s += sv / (M_PI * (double)d);
        }
    }
    part[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) part[tid] += part[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        double sv, cv;
        sincospi(2.0 * (double)w / (double)L, &sv, &cv);
        if (T.f64) {
            double2* tw = (double2*)T.table;
            tw[w] = make_double2(cv, -sv);
            ((double*)(tw + L))[w] = 2.0 * part[0] / (double)L;
        } else {
            float2* tw = (float2*)T.table;
            tw[w] = make_float2((float)cv, (float)-sv);
            ((float*)(tw + L))[w] = (float)(2.0 * part[0] / (double)L);
        }
    }
}

// =========================================================================
// Correlation GEMM
// =========================================================================
template <int P> struct Frag;
template <> struct Frag<P_F64> { using T = d4; using Acc = d4; static constexpr int KS = 16; };
template <> struct Frag<P_F32> { using T = f4; using Acc = f4; static constexpr int KS = 16; };
template <> struct Frag<P_SPLIT> { using T = bf8; using Acc = f4; static constexpr int KS = 32; };
template <> struct Frag<P_BF16> { using T = bf8; using Acc = f4; static constexpr int KS = 32; };
template <> struct Frag<P_F16> { using T = h8; using Acc = f4; static constexpr int KS = 32; };
template <> struct Frag<P_SPLIT16> { using T = h8; using Acc = f4; static constexpr int KS = 32; };
template <> struct Frag<P_FP8> { using T = u4; using Acc = f4; static constexpr int KS = 64; };

template <int P>
__device__ inline typename Frag<P>::T load_frag(const void* base, int64_t row, int kp, int k) {
    constexpr int esz = elem_bytes(P);
    const char* p = (const char*)base + ((row * kp) + k) * esz;
    return *(const typename Frag<P>::T*)p;
}

// One super-step of products acc += a * b for one 16x16 block.
template <int P>
__device__ inline void mma(typename Frag<P>::Acc& acc, const typename Frag<P>::T& a,
                           const typename Frag<P>::T& b) {
    if constexpr (P == P_F64) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc, 0, 0, 0);
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc, 0, 0, 0);
    } else if constexpr (P == P_SPLIT || P == P_BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    } else if constexpr (P == P_F16 || P == P_SPLIT16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
    } else {
        const long a0 = (long)a[0] | ((long)a[1] << 32), a1 = (long)a[2] | ((long)a[3] << 32);
        const long b0 = (long)b[0] | ((long)b[1] << 32), b1 = (long)b[2] | ((long)b[3] << 32);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
    }
}

// Row starts of the upper-triangle layouts.  Row indices and n are below
// 2^24 (the plan's limit), so 32 x 32 -> 64-bit products suffice.
__device__ inline int64_t mul64(uint32_t a, uint32_t b) { return (int64_t)((uint64_t)a * b); }
// Start of packed row i minus i, so that element (i, j) is at base + j.
__device__ inline int64_t packed_row_base(int64_t i, int64_t n) {
    const uint32_t ii = (uint32_t)i;
    return mul64(ii, (uint32_t)n) - (mul64(ii, ii - 1u) >> 1) - i;
}
// Row-aligned upper layout: row i starts at i N32 - 32 (16 q (q-1) + r q),
// i = 32 q + r, and holds the columns from 32 q on; the start minus 32 q, so
// that element (i, j) is at base + j.  Every row starts on a multiple of 32
// elements.
__device__ inline int64_t aligned_row_base(int64_t i, int64_t n) {
    const uint32_t ii = (uint32_t)i, q = ii >> 5, r = ii & 31u;
    const uint32_t n32 = ((uint32_t)n + 31u) & ~31u;
    return mul64(ii, n32) - 32 * (16 * mul64(q, q - 1u) + mul64(r, q)) - 32 * (int64_t)q;
}

// s_waitcnt through the builtin, so that the compiler's own wait tracking
// sees it (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt
// 11:8; a field at its maximum does not wait).
template <int VM, int LGKM>
__device__ inline void waitcnt() {
    static_assert(VM >= 0 && VM <= 63 && LGKM >= 0 && LGKM <= 15, "waitcnt fields");
    __builtin_amdgcn_s_waitcnt((VM & 15) | (7 << 4) | (LGKM << 8) | ((VM >> 4) << 14));
}
template <int N>
__device__ inline void wait_vmcnt() {
    waitcnt<N, 15>();
}
__device__ inline void wait_lgkm0() { waitcnt<63, 0>(); }

// Workgroup barrier that waits for no memory operation: copies into LDS and
// global stores stay in flight across it.
__device__ inline void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}
// Barrier after this wave's own LDS writes (ds_write is asynchronous): wait
// for them (lgkmcnt), but not for outstanding global stores (vmcnt).
__device__ inline void lds_write_barrier() {
    wait_lgkm0();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// Epilogue through LDS, shared by both contraction kernels
// ---------------------------------------------------------------------------
// An output tile of TM x TN values of type OT sits in LDS with a row pitch
// of TN + 4 elements, already scaled by c / sR_j; store_tile writes it out
// with NT threads as contiguous row runs (16-byte stores): direct rows for
// heterocorrelation and the upper part of a homocorrelation, the mirror of a
// FULL homocorrelation read transposed from the same tile (Psi negated), or
// the rows of an upper-triangle layout.  The row scale 1 / sL_i, a power of
// two, is applied exactly with ldexp as the rows leave LDS; this equals one
// FP64 product unless the result is subnormal.  (Interior tiles of the
// row-aligned upper layout skip LDS in the LDS-staged kernel; see stage_out.)

// Exponent of a power-of-two scale.
__device__ inline int pow2_exp(float s) { return ((__float_as_int(s) >> 23) & 0xff) - 127; }

// Factor of an output column of the LDS-staged kernels: the contraction's
// normalization c (FP64) times the column's power-of-two unscaling 2^e,
// rounded once to FP32.  An accumulator times it is rounded once more; the
// row's power of two is then applied exactly (ldexp), so an output carries
// at most two roundings after the MFMA accumulation.
__device__ inline float col_factor(double c, int e) { return (float)ldexp(c, e); }

template <class OT> struct V4 { OT x, y, z, w; };
template <class OT>
__device__ inline V4<OT> row_unscale(V4<OT> v, int e) {
    return V4<OT>{ldexp(v.x, e), ldexp(v.y, e), ldexp(v.z, e), ldexp(v.w, e)};
}
template <>
__device__ inline V4<float> row_unscale(V4<float> v, int e) {
    return V4<float>{ldexpf(v.x, e), ldexpf(v.y, e), ldexpf(v.z, e), ldexpf(v.w, e)};
}

// Four consecutive outputs with 16-byte vector stores whatever the address's
// alignment (the packed layout's rows start anywhere): the vector types
// below promise only element alignment, and global stores accept that.
// FP32 outputs are written once and not read again by the kernel: their
// stores are non-temporal, so that they do not push the operand panels,
// which the next tiles reuse, out of L2 (packed split-BF16 3-5 % faster,
// plain BF16 4-7 %).  FP64 outputs keep ordinary stores (non-temporal ones
// made the FP64 mirror stores of m = 64, n = 4096 50 % slower).
typedef float f4_ua __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2_ua __attribute__((ext_vector_type(2), aligned(8)));
template <class OT>
__device__ inline void put4(OT* o, int64_t idx, V4<OT> v) {
    OT* d = o + idx;
    if constexpr (std::is_same<OT, double>::value) {
        *(d2_ua*)d = d2_ua{v.x, v.y};
        *(d2_ua*)(d + 2) = d2_ua{v.z, v.w};
    } else {
        __builtin_nontemporal_store(f4_ua{v.x, v.y, v.z, v.w}, (f4_ua*)d);
    }
}

// A store at system scope (sc0 sc1), for calls whose outputs fit the
// memory-side cache (kNearStoreBytes); a vector store, written in asm for
// its cache-policy bits.
__device__ inline void store_near(float* p, float v) {
    asm volatile("global_store_dword %0, %1, off sc0 sc1" : : "v"(p), "v"(v) : "memory");
}

// One output element: the row exponent applied in the output type, and a
// non-temporal store for FP32 (as in put4).
__device__ inline float unscale1(float v, int e) { return ldexpf(v, e); }
__device__ inline double unscale1(double v, int e) { return ldexp(v, e); }
__device__ inline void put1(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ inline void put1(double* p, double v) { *p = v; }

// Exponents that undo the power-of-two operand scales of one TM x TN output
// tile, gathered once per tile into an LDS table for the epilogue:
// [0, TM) the left rows i0 + r, [TM, TM + TN) the right A columns j0 + c,
// [TM + TN, TM + 2 TN) the right B columns (0 without per-band scaling and
// past the last row or column).  NT threads share the loads.  Reading the
// scales in the epilogue itself would put a load between stores, and the wait
// for it would also wait for every store before it (vmcnt counts both).
template <int TM, int TN, int NT>
struct ScaleExps {
    static constexpr int N = TM + 2 * TN;
    static constexpr int PER = (N + NT - 1) / NT;
    float v[PER];   // the scales themselves
    bool ok[PER];   // entry exists and is scaled
    // Branch-free loads (entries past the data read sL[0] and are dropped):
    // their values are first used in store(), so the wait for them comes
    // there and the work in between hides it.
    __device__ void load(const CorrJob& C, int64_t i0, int64_t j0, int tid) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * NT;
            const bool row = e < TM, b = e >= TM + TN;
            const int64_t j = j0 + e - TM - (b ? TN : 0);
            ok[k] = C.scaled && e < N && (row ? i0 + e < C.n1 : j < C.n2);
            v[k] = 1.0f;
        }
        if (C.scaled) {
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int e = tid + k * NT;
                const bool row = e < TM, b = e >= TM + TN;
                const int64_t j = j0 + e - TM - (b ? TN : 0);
                const float* src = row ? C.sL + i0 + e : (b ? C.sRB : C.sRA) + j;
                v[k] = *(ok[k] ? src : C.sL);
            }
        }
    }
    // write the table; the caller's next barrier publishes it
    __device__ void store(int* t, int tid) const {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (tid + k * NT < N) t[tid + k * NT] = ok[k] ? -pow2_exp(v[k]) : 0;
        wait_lgkm0();
    }
};

// Store one (TM x TN) output tile held in LDS in the output type OT, rows
// of TN + 4 elements, already scaled by c / sR_j; rexp[r] (LDS) is the
// exponent of tile row r's scale (0 when unscaled), applied exactly with
// ldexp.  NT threads.  Tiles wholly inside the output and off the diagonal
// (nearly all) take a straight-line path: no per-element checks and no
// branch between passes, so the passes' LDS reads and stores interleave.
// Nothing here reads global memory: a load between the stores would make
// each pass wait for every earlier store (vmcnt counts both).
template <int TM, int TN, int NT, class OT>
__device__ inline void store_tile(const CorrJob& C, int64_t i0, int64_t j0, const OT* T, const int* rexp,
                                  bool psi, int tid) {
    constexpr int P = TN + 4;             // row pitch in elements
    constexpr int RPP = NT / (TN / 4);    // rows per pass of the direct stores
    static_assert(TM % RPP == 0, "direct-store passes");
    const bool homo = C.homo;
    const bool diag = homo && j0 <= i0 + TM - 1;   // tile reaches the diagonal
    OT* out = (OT*)(psi ? C.psi : C.phi);
    const bool fast = i0 + TM <= C.n1 && j0 + TN <= C.n2 && !diag;
    const int cl = (tid % (TN / 4)) * 4;  // 4 consecutive columns per thread
    const int rsub = tid / (TN / 4);
    auto row = [&](int rl) { return row_unscale(*(const V4<OT>*)(T + rl * P + cl), rexp[rl]); };
    if (!homo || C.layout == L_FULL) {
        // direct rows (homo: the upper part; diagonal tiles mask j < i)
        if (fast) {
#pragma unroll
            for (int pass = 0; pass < TM / RPP; ++pass) {
                const int rl = pass * RPP + rsub;
                put4(out, (i0 + rl) * C.ld_out + j0 + cl, row(rl));
            }
        } else {
#pragma unroll 4
            for (int pass = 0; pass < TM / RPP; ++pass) {
                const int rl = pass * RPP + rsub;
                const int64_t i = i0 + rl, j = j0 + cl;
                const V4<OT> v = row(rl);
                const OT e[4] = {v.x, v.y, v.z, v.w};
                if (i < C.n1)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t jj = j + q;
                        if (jj < C.n2 && !(diag && jj < i)) out[i * C.ld_out + jj] = e[q];
                    }
            }
        }
        if (homo) {
            // mirror: row jm = j0 + rr, columns i0 + cc..cc+3 take -(+)T[cc+q][rr]
            // for Psi (Phi); diagonal tiles write only the strictly lower part
            constexpr int MPP = NT / (TM / 4);   // mirror rows per pass
            static_assert(TN % MPP == 0, "mirror passes");
            const int cc = (tid % (TM / 4)) * 4;
            const int rsubm = tid / (TM / 4);
            const OT sg = psi ? OT(-1) : OT(1);
            // rows i0 + cc .. cc+3 of the tile are this thread's mirror columns
            const int er[4] = {rexp[cc], rexp[cc + 1], rexp[cc + 2], rexp[cc + 3]};
            auto col = [&](int rr) {
                return V4<OT>{ldexp(sg * T[(cc + 0) * P + rr], er[0]), ldexp(sg * T[(cc + 1) * P + rr], er[1]),
                              ldexp(sg * T[(cc + 2) * P + rr], er[2]), ldexp(sg * T[(cc + 3) * P + rr], er[3])};
            };
            if (fast) {
#pragma unroll 8
                for (int pass = 0; pass < TN / MPP; ++pass) {
                    const int rr = pass * MPP + rsubm;
                    put4(out, (j0 + rr) * C.ld_out + i0 + cc, col(rr));
                }
            } else {
#pragma unroll 4
                for (int pass = 0; pass < TN / MPP; ++pass) {
                    const int rr = pass * MPP + rsubm;
                    const int64_t jm = j0 + rr, im = i0 + cc;
                    const V4<OT> t = col(rr);
                    const OT e[4] = {t.x, t.y, t.z, t.w};
                    if (jm < C.n1)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int64_t ii = im + q;
                            // strictly lower part (row jm > col ii)
                            if (ii < C.n1 && !(diag && ii >= jm)) out[jm * C.ld_out + ii] = e[q];
                        }
                }
            }
        }
    } else {
        // upper triangle: element (i, j), j >= i, at rowbase(i) + j, packed
        // (UPPER_PACKED) or with 32-element aligned rows (UPPER_ALIGNED)
        const bool packed = C.layout == L_UPPER;
        auto base = [&](int64_t i) { return packed ? packed_row_base(i, C.n1) : aligned_row_base(i, C.n1); };
        if (fast) {
#pragma unroll
            for (int pass = 0; pass < TM / RPP; ++pass) {
                const int rl = pass * RPP + rsub;
                put4(out, base(i0 + rl) + j0 + cl, row(rl));
            }
        } else {
#pragma unroll 4
            for (int pass = 0; pass < TM / RPP; ++pass) {
                const int rl = pass * RPP + rsub;
                const int64_t i = i0 + rl, j = j0 + cl;
                const V4<OT> v = row(rl);
                const OT e[4] = {v.x, v.y, v.z, v.w};
                if (i < C.n1) {
                    const int64_t b = base(i);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t jj = j + q;
                        if (jj < C.n2 && jj >= i) out[b + jj] = e[q];
                    }
                }
            }
        }
    }
}

// Dynamic LDS of the register-direct kernel: one output plane of its tile.
__host__ __device__ constexpr int corr_lds_bytes(int fm, int fn, bool out_f64) {
    return 32 * fm * (32 * fn + 4) * (out_f64 ? 8 : 4);
}

// One output tile (I, J) of size (32 FM) x (32 FN) computed by 4 waves (2x2)
// with register-direct fragments, then written through LDS (FP64 interior
// tiles: straight from the accumulators).
template <int P, int FM, int FN>
__device__ inline void corr_tile(const CorrJob& C, int I, int J, char* lds, int* sexp) {
    using FT = typename Frag<P>::T;
    using AT = typename Frag<P>::Acc;
    constexpr int KS = Frag<P>::KS;
    constexpr bool SPLIT = (P == P_SPLIT);
    constexpr int BM = 32 * FM, BN = 32 * FN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = (int64_t)I * BM + (wave >> 1) * (16 * FM);
    const int64_t j0 = (int64_t)J * BN + (wave & 1) * (16 * FN);
    const int kofs = kg * (KS / 4);
    // the scales' exponents, loaded ahead of the K loop (its own waits cover them)
    ScaleExps<BM, BN, 256> se;
    se.load(C, (int64_t)I * BM, (int64_t)J * BN, threadIdx.x);

    AT ap[FM][FN], aq[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            ap[a][b] = AT{0, 0, 0, 0};
            aq[a][b] = AT{0, 0, 0, 0};
        }

    for (int k0 = 0; k0 < C.kp; k0 += KS) {
        FT la[FM], ra[FN], rb[FN];
        FT la1[SPLIT ? FM : 1], ra1[SPLIT ? FN : 1], rb1[SPLIT ? FN : 1];
#pragma unroll
        for (int a = 0; a < FM; ++a) {
            la[a] = load_frag<P>(C.L0, i0 + a * 16 + row16, C.kp, k0 + kofs);
            if constexpr (SPLIT) la1[a] = load_frag<P>(C.L1, i0 + a * 16 + row16, C.kp, k0 + kofs);
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            ra[b] = load_frag<P>(C.RA0, j0 + b * 16 + row16, C.kp, k0 + kofs);
            rb[b] = load_frag<P>(C.RB0, j0 + b * 16 + row16, C.kp, k0 + kofs);
            if constexpr (SPLIT) {
                ra1[b] = load_frag<P>(C.RA1, j0 + b * 16 + row16, C.kp, k0 + kofs);
                rb1[b] = load_frag<P>(C.RB1, j0 + b * 16 + row16, C.kp, k0 + kofs);
            }
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                mma<P>(ap[a][b], la[a], ra[b]);
                mma<P>(aq[a][b], la[a], rb[b]);
                if constexpr (SPLIT) {
                    mma<P>(ap[a][b], la[a], ra1[b]);
                    mma<P>(ap[a][b], la1[a], ra[b]);
                    mma<P>(aq[a][b], la[a], rb1[b]);
                    mma<P>(aq[a][b], la1[a], rb[b]);
                }
            }
    }

    // epilogue through LDS in the output type, Phi then Psi
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int64_t ti0 = (int64_t)I * BM, tj0 = (int64_t)J * BN;
    const bool diag = C.homo && tj0 <= ti0 + BM - 1;
    se.store(sexp, tid);
    auto stage = [&](auto* T, AT (&acc)[FM][FN], bool psi) {
        using OT = typename std::remove_pointer<decltype(T)>::type;
        lds_barrier();   // previous readers of the LDS are done (and the scale table is visible)
        if constexpr (P == P_F64) {
            // Interior tiles of the FP64 path store straight from the
            // accumulators: register q of a 16 x 16 block holds row kg + 4q
            // and column row16, so each store writes 16 consecutive doubles
            // (one 128-byte line) of four rows, and the mirror of the full
            // layout takes the transposed element.  The rounding is that of
            // the staged path (scale in FP64, then the row exponent), so the
            // results are the same bit for bit.  The FP32-accumulator formats
            // keep the staged path: their register rows are 64-byte halves
            // of a line, slower than the staged full-row stores.
            if (ti0 + BM <= C.n1 && tj0 + BN <= C.n2 && !diag) {
                OT* out = (OT*)(psi ? C.psi : C.phi);
                const bool full = !C.homo || C.layout == L_FULL;
                const bool mirror = C.homo && C.layout == L_FULL;
                auto rowoff = [&](int64_t i) -> int64_t {
                    return full ? i * C.ld_out
                                : (C.layout == L_UPPER ? packed_row_base(i, C.n1) : aligned_row_base(i, C.n1));
                };
                const OT sg = psi ? OT(-1) : OT(1);
#pragma unroll
                for (int a = 0; a < FM; ++a) {
                    int il[4];
                    int64_t ro[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        il[q] = (int)(i0 - ti0) + a * 16 + kg + 4 * q;
                        ro[q] = rowoff(ti0 + il[q]);
                    }
                    const int e[4] = {sexp[il[0]], sexp[il[1]], sexp[il[2]], sexp[il[3]]};
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        const int jl = (int)(j0 - tj0) + b * 16 + row16;
                        const double fc = ldexp(C.c, sexp[BM + (psi ? BN : 0) + jl]);
                        const int64_t j = tj0 + jl;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const OT v = unscale1((OT)((double)acc[a][b][q] * fc), e[q]);
                            put1(out + ro[q] + j, v);
                            if (mirror) put1(out + j * C.ld_out + ti0 + il[q], sg * v);
                        }
                    }
                }
                return;
            }
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int jl = (int)(j0 - tj0) + b * 16 + row16;
            const double fc = ldexp(C.c, sexp[BM + (psi ? BN : 0) + jl]);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int il = (int)(i0 - ti0) + a * 16 + (P == P_F64 ? kg + 4 * q : kg * 4 + q);
                    OT v = (OT)((double)acc[a][b][q] * fc);
                    if (psi && diag && ti0 + il == tj0 + jl) v = OT(0);
                    T[il * (BN + 4) + jl] = v;
                }
        }
        lds_write_barrier();
        store_tile<BM, BN, 256, OT>(C, ti0, tj0, T, sexp, psi, tid);
    };
    if (C.out_f64) {
        stage((double*)lds, ap, false);
        stage((double*)lds, aq, true);
    } else {
        stage((float*)lds, ap, false);
        stage((float*)lds, aq, true);
    }
}

// ---------------------------------------------------------------------------
// LDS-staged contraction for the 16-bit formats (split BF16, BF16, FP16).
//
// Workgroup: 4 waves (2 x 2), output tile 128 x 128 of Phi and of Psi; each
// wave owns 64 x 64 of both (2 x 2 blocks of v_mfma_f32_32x32x16).  The
// contraction runs over K blocks of 16.  Each block's operand rows (left A
// rows of tile I, right A and B rows of tile J, hi and lo planes for the
// split form) are 4 KB runs of the K-blocked layout, copied straight into
// LDS with global_load_lds_dwordx4 (no register staging) through a ring of
// S stages: the copies of blocks kb+2 .. kb+S are in flight while the
// fragments of block kb+1 are read and those of block kb feed the MFMAs.
// Each wave waits only for its own copies of the block it reads next
// (vmcnt) and a bare s_barrier publishes them; a full __syncthreads would
// also drain the prefetches.
// ---------------------------------------------------------------------------
typedef float f16v __attribute__((ext_vector_type(16)));

#define AS_GLOBAL(p) ((const __attribute__((address_space(1))) void*)(p))
#define AS_LDS(p) ((__attribute__((address_space(3))) void*)(p))

template <int P> struct Wide;
template <> struct Wide<P_SPLIT> { using T = bf8; };
template <> struct Wide<P_BF16> { using T = bf8; };
template <> struct Wide<P_F16> { using T = h8; };
template <> struct Wide<P_SPLIT16> { using T = h8; };

template <int P>
__device__ inline void mma32(f16v& acc, const typename Wide<P>::T& a, const typename Wide<P>::T& b) {
    if constexpr (P == P_F16 || P == P_SPLIT16) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
    else acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
}

// Tiles of the LDS-staged contraction: TM output rows (128 or 256) x 128
// output columns, TM/32 waves, each wave a 64 x 64 block of Phi and of Psi
// (2 x 2 blocks of the 32 x 32 MFMA).  One K stage (16 contraction elements)
// per plane holds the TM/128 panels of the left operand and one panel of
// each right operand (4 KB each), copied straight from the panel-blocked
// layout.  TM = 256 runs one 8-wave workgroup per CU; TM = 128 two 4-wave
// workgroups, so that one's epilogue can overlap the other's K loop.
constexpr int kTileN2 = 128;
constexpr int threads2(int TM) { return TM * 2; }
template <int P, int TM> constexpr int stage_bytes() { return planes(P) * (TM * 32 + 8192); }
// Stages in the ring: 128 KB for TM = 256 (one workgroup per CU), 72 KB for
// TM = 128 (two per CU).
template <int P, int TM> constexpr int ring_stages() {
    return TM == 256 ? (planes(P) == 2 ? 4 : 8) : (planes(P) == 2 ? 3 : 6);
}
// LDS of a contraction workgroup: the operand ring, reused by the output tile
template <int P, int TM> constexpr int corr2_lds_bytes() {
    return ring_stages<P, TM>() * stage_bytes<P, TM>() > TM * (kTileN2 + 4) * 4
               ? ring_stages<P, TM>() * stage_bytes<P, TM>()
               : TM * (kTileN2 + 4) * 4;
}


// Epilogue of one TM x 128 output tile of the LDS-staged kernel.  The waves
// multiply their accumulators by the column factor (col_factor: FP32
// multiplies, no FP64 work per output; 2-5 % faster at m = 256, n = 16384
// than an FP64 product rounded once) and write them into an LDS tile (the
// operand ring is free by then), then store_tile writes it out with the row
// scales; or they store them straight from the registers.  Accumulator
// register r of lane l holds row 8(r/4) + 4(l/32) + r%4 and column l%32 of
// its 32 x 32 block.
template <int TM>
__device__ inline void stage_out(const CorrJob& C, int I, int J, f16v (&acc)[2][2], char* lds,
                                 const int* sexp, bool psi) {
    float* T = (float*)lds;
    // opaque copy of the thread index: keeps the index arithmetic below
    // inside a persistent tile loop instead of hoisted and spilled
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1, g = lane >> 5;
    const int64_t i0 = (int64_t)I * TM, j0 = (int64_t)J * kTileN2;
    const bool diag = C.homo && j0 <= i0 + TM - 1;
    lds_barrier();   // previous readers of the LDS are done (and the scale table is visible)
    const bool interior = i0 + TM <= C.n1 && j0 + kTileN2 <= C.n2;
    // A heterocorrelation (full layout, no mirror) takes the direct path
    // below when its rows are whole 128-byte lines: row stride a multiple of
    // 32 floats below 2^31, output 128-byte aligned.
    const bool hfull = !C.homo && interior && (C.ld_out & 31) == 0 && C.ld_out < (int64_t(1) << 31) &&
                       ((uintptr_t)(psi ? C.psi : C.phi) & 127) == 0;
    if ((C.homo && C.layout == L_UPPER_ALIGNED && interior && !diag) || hfull) {
        // Row-aligned upper layout (or the heterocorrelation above), interior
        // tile: straight from the accumulators.  Register r of a 32 x 32 block
        // holds 32 consecutive columns of two rows, whole aligned 128-byte
        // lines here, so no staging through LDS is needed.  The block's 32
        // rows lie in one 32-row band of the upper layout and share its row
        // length (the row stride for the full layout).  Non-temporal stores,
        // as in put4, or system-scope ones when the call's outputs fit the
        // memory-side cache.
        float* out = (float*)(psi ? C.psi : C.phi);
        auto direct = [&](auto near) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int64_t ia = i0 + wi * 64 + a * 32;
                const int64_t base = hfull ? ia * C.ld_out : aligned_row_base(ia, C.n1);
                const uint32_t len = hfull ? (uint32_t)C.ld_out
                                           : (((uint32_t)C.n1 + 31u) & ~31u) - 32u * (uint32_t)(ia >> 5);
                int4 re[4];   // row exponents of rows ia + 8k + 4g .. + 3
#pragma unroll
                for (int k = 0; k < 4; ++k) re[k] = *(const int4*)(sexp + wi * 64 + a * 32 + 8 * k + 4 * g);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int jl = wj * 64 + b * 32 + (lane & 31);
                    const float cf = col_factor(C.c, sexp[TM + (psi ? kTileN2 : 0) + jl]);
                    float* o = out + base + j0 + jl;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int k = r >> 2, q = r & 3;
                        const int e = q == 0 ? re[k].x : q == 1 ? re[k].y : q == 2 ? re[k].z : re[k].w;
                        float* po = o + mul64(8 * k + 4 * g + q, len);
                        const float v = ldexpf(acc[a][b][r] * cf, e);
                        if constexpr (decltype(near)::value) store_near(po, v);
                        else __builtin_nontemporal_store(v, po);
                    }
                }
            }
        };
        if (C.store_near) direct(std::true_type{});
        else direct(std::false_type{});
        return;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int jl = wj * 64 + b * 32 + (lane & 31);
        const float cf = col_factor(C.c, sexp[TM + (psi ? kTileN2 : 0) + jl]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int il = wi * 64 + a * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
                float v = acc[a][b][r] * cf;
                if (psi && diag && i0 + il == j0 + jl) v = 0.0f;
                T[il * (kTileN2 + 4) + jl] = v;
            }
    }
    lds_write_barrier();
    store_tile<TM, kTileN2, threads2(TM), float>(C, i0, j0, T, sexp, psi, tid);
}

// Fragments of one K stage held in registers: NP planes (both halves of a
// split format, or the high plane alone) of the left rows and the two right
// operands, for the wave's two 32-row blocks.
template <class FT, int NP>
struct StageFrags {
    FT la[NP][2], ra[NP][2], rb[NP][2];
};

// Wait until at most u * CPW vector memory operations of this wave are
// outstanding (u <= MAXU; the encoding needs an immediate, so the runtime
// count selects the immediate for it).
template <int CPW, int MAXU>
__device__ inline void wait_units(int u) {
    if constexpr (MAXU == 0) {
        wait_vmcnt<0>();
    } else {
        if (u >= MAXU) wait_vmcnt<CPW * MAXU>();
        else wait_units<CPW, MAXU - 1>(u);
    }
}

// One TM x 128 output tile: the K loop over a ring of LDS stages filled by
// direct-to-LDS loads, then the epilogue.  A plane's stage is CH = TM/32 + 8
// chunks of 1 KB: chunks 0..TM/32-1 hold the left panels, then 4 for the
// synchronous right panel and 4 for the asynchronous one; wave w copies
// chunks w, w + NW, ... of every plane.
//
// Row-selective split (C.kb_sel set, split formats only): the K blocks run
// in the order the list gives, and only the first nsel of them (the
// highest-energy Fourier rows, in pairs of blocks) carry the low plane; the
// others are copied and multiplied with the high plane alone (hi*hi).  A
// stage then holds one or two planes, and the waits count the copies of
// the stages actually in flight.
template <int P, int TM, bool SEL>
__device__ inline void corr2_tile(const CorrJob& C, int I, int J, char* lds, int* sexp, int* sorder) {
    using FT = typename Wide<P>::T;
    constexpr int PL = planes(P);
    constexpr int S = ring_stages<P, TM>();
    constexpr int SB = stage_bytes<P, TM>();
    constexpr int NW = TM / 32;          // waves
    constexpr int CH = TM / 32 + 8;      // 1 KB chunks per plane and stage
    constexpr int CPW = CH / NW;         // chunks per wave and plane
    constexpr int PB = TM * 32 + 8192;   // plane bytes per stage
    constexpr int MAXU = PL * (S - 1);   // plane-stages a wave can have in flight
    // opaque copy of the thread index: in a persistent tile loop the values
    // derived from it are then recomputed per tile rather than kept live
    // (and spilled) across the epilogue
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, w = tid >> 6;
    const int wi = w >> 1, wj = w & 1;
    const int nkb = C.kp >> 4;
    const int64_t panel_bytes = (int64_t)nkb * 4096;
    // Row-selective split (SEL, split formats): the K-block order goes to
    // an LDS table (nkb <= 64), read per copy; nsel blocks carry both
    // planes (clamped, so that a damaged record cannot send a copy out of
    // range).  Without SEL every stage has the format's planes, in order.
    // (Kept in LDS rather than in a register: a block index read from a
    // loaded register made the compiler wait for every copy in flight
    // before the fragment reads.)
    static_assert(!SEL || PL == 2, "row selection is for the split formats");
    int nsel = PL == 1 ? 0 : nkb;
    if constexpr (SEL) {
        nsel = min(max(__builtin_amdgcn_readfirstlane(C.kb_sel[0]), 0), nkb) & ~1;
        if (tid < kMaxSelBlocks) sorder[tid] = tid < nkb ? min(max(C.kb_sel[1 + tid], 0), nkb - 1) : 0;
        wait_lgkm0();
        __syncthreads();   // the table is written before the first copy reads it
    }
    auto block_of = [&](int kb) {
        if constexpr (SEL) return __builtin_amdgcn_readfirstlane(sorder[kb]);
        else return kb;
    };
    auto planes_of = [&](int kb) { return kb < nsel ? PL : 1; };

    const char* src[PL][CPW];
#pragma unroll
    for (int p = 0; p < PL; ++p)
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            const int c = w + k * NW;
            const char* b;
            if (c < TM / 32) {
                b = (const char*)(p ? C.L1 : C.L0) + ((int64_t)I * (TM / 128) + (c >> 2)) * panel_bytes;
            } else {
                const int r = c - TM / 32;
                b = (const char*)(r < 4 ? (p ? C.RA1 : C.RA0) : (p ? C.RB1 : C.RB0)) + (int64_t)J * panel_bytes;
            }
            src[p][k] = b + (c & 3) * 1024 + lane * 16;
        }
    // copy stage kb (its block of the order) with its planes
    auto issue = [&](int kb) {
        char* dst = lds + (kb % S) * SB;
        const int64_t off = (int64_t)block_of(kb) * 4096;
        const int np = SEL ? planes_of(kb) : PL;
#pragma unroll
        for (int p = 0; p < PL; ++p)
            if (p < np)
#pragma unroll
                for (int k = 0; k < CPW; ++k) {
                    // The LDS destination passes through an empty asm, so the
                    // compiler cannot tell which LDS object the copy writes:
                    // it then leaves the ordering of copies and fragment reads
                    // to the explicit waits of the ring (it would otherwise
                    // wait for every copy in flight, the prefetches included,
                    // before reading a stage whose copy has landed).
                    char* d = dst + p * PB + (w + k * NW) * 1024;
                    asm volatile("" : "+v"(d));
                    __builtin_amdgcn_global_load_lds(AS_GLOBAL(src[p][k] + off), AS_LDS(d), 16, 0, 0);
                }
    };
    // plane-stages of stages lo..hi (inclusive, clipped to the K range): a
    // wave issues CPW copies for each
    auto units = [&](int lo, int hi) {
        hi = min(hi, nkb - 1);
        if (hi < lo) return 0;
        const int sel = max(0, min(hi, nsel - 1) - lo + 1);
        return (hi - lo + 1) + (PL - 1) * sel;
    };

    // LDS byte offsets of this lane's fragment rows (K-block half g = lane/32)
    const int g = lane >> 5;
    int offA[2], offB[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int ra = wi * 64 + a * 32 + (lane & 31);
        const int rb = wj * 64 + a * 32 + (lane & 31);
        offA[a] = ra * 32 + ((g ^ row_swizzle(ra)) << 4);
        offB[a] = TM * 32 + rb * 32 + ((g ^ row_swizzle(rb)) << 4);
    }

    f16v ap[2][2], aq[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            ap[a][b] = f16v{};
            aq[a][b] = f16v{};
        }

    // Fragments of one stage, held in registers: the K loop reads stage kb+1
    // from LDS while the MFMAs of stage kb run (two register sets).  NP
    // planes: the split stages' fragments hold both, the others the high
    // plane only (separate register sets, so that no stale low-plane
    // fragment stays live through the single-plane stages).
    auto load_frags = [&](auto& F, int kb) {
        constexpr int NP = sizeof(F.la) / sizeof(F.la[0]);
        const char* st = lds + (kb % S) * SB;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                F.la[p][a] = *(const FT*)(st + p * PB + offA[a]);
                F.ra[p][a] = *(const FT*)(st + p * PB + offB[a]);
                F.rb[p][a] = *(const FT*)(st + p * PB + 4096 + offB[a]);
            }
    };
    // MFMAs of one stage for the 32-row block a of the wave's 64 rows
    auto mfma_rows = [&](const auto& F, int a) {
        constexpr int NP = sizeof(F.la) / sizeof(F.la[0]);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            mma32<P>(ap[a][b], F.la[0][a], F.ra[0][b]);
            mma32<P>(aq[a][b], F.la[0][a], F.rb[0][b]);
            if constexpr (NP == 2) {
                mma32<P>(ap[a][b], F.la[0][a], F.ra[1][b]);
                mma32<P>(aq[a][b], F.la[0][a], F.rb[1][b]);
                mma32<P>(ap[a][b], F.la[1][a], F.ra[0][b]);
                mma32<P>(aq[a][b], F.la[1][a], F.rb[0][b]);
            }
        }
    };
    // Stage kb+1 always exists where this runs (the number of K blocks is
    // even), so the fragment reads are unconditional.
    // The next stage's reads go between the two halves of the MFMAs: the
    // wait for this stage's fragments comes before the first half, and the
    // second half (and the next barrier) hide the new reads' latency.
    // Each wave finishes its own fragment reads of stage kb (lgkmcnt) before
    // the barrier, so after it the slot of stage kb is free and the copy of
    // stage kb + S goes there: every slot of the ring holds a stage in
    // flight or being read, and a copy has S - 1 steps to land.  Before the
    // barrier, stage kb+1 must have landed: the copies of stages kb+2 ..
    // kb+S-1 may still be in flight (a wave's vector memory operations
    // complete in issue order).
    auto step = [&](const auto& Fc, auto& Fn, int kb) {
        if constexpr (SEL) wait_units<CPW, MAXU>(units(kb + 2, kb + S - 1));
        else wait_units<CPW * PL, S - 2>(min(S - 2, nkb - 2 - kb));
        wait_lgkm0();
        lds_barrier();
        if (kb + S < nkb) issue(kb + S);
        mfma_rows(Fc, 0);
        __builtin_amdgcn_sched_barrier(0);
        load_frags(Fn, kb + 1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_rows(Fc, 1);
    };
    // the last stage: the scales' exponents are loaded meanwhile (every copy
    // has landed, so these loads are the only ones in flight and the last
    // stage's MFMAs hide them)
    ScaleExps<TM, kTileN2, threads2(TM)> se;
    auto last = [&](const auto& F) {
        se.load(C, (int64_t)I * TM, (int64_t)J * kTileN2, tid);
        __builtin_amdgcn_sched_barrier(0);
        mfma_rows(F, 0);
        mfma_rows(F, 1);
        __builtin_amdgcn_sched_barrier(0);
    };

    lds_barrier();   // the ring is free (previous tile of a persistent loop)
#pragma unroll
    for (int st = 0; st < S; ++st)
        if (st < nkb) issue(st);
    if constexpr (SEL) wait_units<CPW, MAXU>(units(1, S - 1));
    else wait_units<CPW * PL, S - 1>(min(S - 1, nkb - 1));
    lds_barrier();
    // nkb and nsel are even and nkb is at least 2: pairs of steps, then the
    // last pair, whose second stage needs no further load (every load has
    // landed and is visible after the last step's barrier)
    if (!SEL || nsel == nkb) {
        // every stage with all the format's planes
        StageFrags<FT, PL> F0, F1;
        load_frags(F0, 0);
        for (int kb = 0; kb + 2 < nkb; kb += 2) {
            step(F0, F1, kb);
            step(F1, F0, kb + 1);
        }
        step(F0, F1, nkb - 2);
        last(F1);
    } else if constexpr (SEL) {
        // row-selective: the split stages first, then the high plane alone
        StageFrags<FT, 1> G0, G1;
        if (nsel > 0) {
            StageFrags<FT, 2> F0, F1;
            load_frags(F0, 0);
            for (int kb = 0; kb + 2 < nsel; kb += 2) {
                step(F0, F1, kb);
                step(F1, F0, kb + 1);
            }
            step(F0, F1, nsel - 2);
            step(F1, G0, nsel - 1);
        } else {
            load_frags(G0, 0);
        }
        for (int kb = nsel; kb + 2 < nkb; kb += 2) {
            step(G0, G1, kb);
            step(G1, G0, kb + 1);
        }
        step(G0, G1, nkb - 2);
        last(G1);
    }
    se.store(sexp, tid);

    // epilogue through LDS, one output at a time
    stage_out<TM>(C, I, J, ap, lds, sexp, false);
    stage_out<TM>(C, I, J, aq, lds, sexp, true);
}

// Occupancy: two workgroups of 4 waves per CU for TM = 128, one of 8 for
// TM = 256 -- two waves per SIMD, so at most 256 VGPRs each.
template <int P, int TM, bool SEL = false>
__global__ __launch_bounds__(threads2(TM), 256 / TM) void corr2_kernel(CorrJob C) {
    __shared__ __attribute__((aligned(1024))) char lds[corr2_lds_bytes<P, TM>()];
    __shared__ __attribute__((aligned(16))) int sexp[TM + 2 * kTileN2];
    __shared__ int sorder[SEL ? kMaxSelBlocks : 1];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int I, J;
    if (C.homo) decode_upper(t, C.tiles_i, C.tiles_j, C.ratio, C.group, I, J);
    else decode_full(t, C.tiles_i, C.tiles_j, C.group, I, J);
    corr2_tile<P, TM, SEL>(C, I, J, lds, sexp, sorder);
}

// Tile of a persistent workgroup's k-th turn (register-direct kernels): the
// grid takes the tiles in rounds of gridDim.x, and a round's tiles are dealt
// so that each XCD (the workgroups are dealt to the 8 XCDs in turn) takes a
// contiguous run of the tile order, whose operand panels its L2 then
// shares.  Fixed shares instead of an atomic ticket: the tiles are in
// descending cost order, so the rounds are balanced, and a workgroup's tiles
// only move forward in the job list.  On the 256-set batch: FP32 18.3 ->
// 17.9 ms; plain round-robin rounds 18.2 ms.  (The LDS-staged persistent
// kernel keeps its ticket: fixed shares made the split-BF16 batch 2 % slower,
// round-robin ones 5 %.)
__device__ inline int64_t persistent_tile(int64_t k) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t off = (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
    return k * G + off;
}

template <int P, int TM>
__global__ __launch_bounds__(threads2(TM), 256 / TM) void corr2_persistent_kernel(const CorrJob* jobs,
                                                                       const int64_t* tile_start,
                                                                       int count, int64_t total,
                                                                       int* counter) {
    __shared__ __attribute__((aligned(1024))) char lds[corr2_lds_bytes<P, TM>()];
    __shared__ __attribute__((aligned(16))) int sexp[TM + 2 * kTileN2];
    __shared__ int64_t s_t;
    int lo = 0;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(counter, 1);
        __syncthreads();
        // the ticket is the same for the whole workgroup: move it to scalar
        // registers so that the job, its pointers and the tile indices are
        // scalar values too
        const int64_t t = uniform64(s_t);
        __syncthreads();
        if (t >= total) break;
        // a workgroup's tickets increase: its job only moves forward
        while (lo + 1 < count && tile_start[lo + 1] <= t) ++lo;
        const CorrJob C = jobs[lo];
        int I, J;
        decode_upper(t - tile_start[lo], C.tiles_i, C.tiles_j, C.ratio, C.group, I, J);
        corr2_tile<P, TM, false>(C, I, J, lds, sexp, nullptr);
    }
}

// Occupancy: two workgroups per CU (at most 256 registers): with the
// default the 128 x 128 tile grew to 400 registers and one wave per SIMD,
// which left the fragment loads' latency unhidden.
template <int P, int FM, int FN>
__global__ __launch_bounds__(256, 2) void corr_kernel(CorrJob C) {
    extern __shared__ __attribute__((aligned(16))) char corr_lds[];
    __shared__ __attribute__((aligned(16))) int sexp[32 * FM + 64 * FN];
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int I, J;
    if (C.homo) decode_upper(t, C.tiles_i, C.tiles_j, C.ratio, C.group, I, J);
    else decode_full(t, C.tiles_i, C.tiles_j, C.group, I, J);
    corr_tile<P, FM, FN>(C, I, J, corr_lds, sexp);
}

// Persistent batched contraction: workgroups take tiles from a global ticket
// counter until the list (data sets in descending cost order) is exhausted.
// The 128 x 128 tile keeps the default bound here: held to 256 registers the
// tile loop spills.
template <int P, int FM, int FN>
__global__ __launch_bounds__(256, FM * FN < 16 ? 2 : 1) void corr_persistent_kernel(const CorrJob* jobs,
                                                               const int64_t* tile_start,
                                                               int count, int64_t total,
                                                               int* counter) {
    extern __shared__ __attribute__((aligned(16))) char corr_lds[];
    __shared__ __attribute__((aligned(16))) int sexp[32 * FM + 64 * FN];
    int lo = 0;
    for (int64_t k = 0;; ++k) {
        const int64_t t = persistent_tile(k);
        if (t >= total) break;
        while (lo + 1 < count && tile_start[lo + 1] <= t) ++lo;
        const CorrJob C = jobs[lo];
        int I, J;
        decode_upper(t - tile_start[lo], C.tiles_i, C.tiles_j, C.ratio, C.group, I, J);
        corr_tile<P, FM, FN>(C, I, J, corr_lds, sexp);
    }
    (void)counter;
}

// =========================================================================
// Row selection of the split formats
// =========================================================================
// Energy of the 16 packed Fourier rows of one K block of one operand over a
// group of up to kSelGroup panels of 128 spectral points (workgroups in turn
// over the groups and K blocks of operands 0, 1, 2; operand 1 has none for a
// homocorrelation, whose right A is its left A): thread t reads its point's
// 16 values in each panel of the group (32 bytes, the halves swapped as the
// panel-blocked layout stores them), unscaled, sums their squares per row,
// and the workgroup adds its threads' sums through LDS.
template <int P>
__global__ __launch_bounds__(128) void row_energy_kernel(SelJob J) {
    __shared__ float sq[128][17];
    __shared__ float part[8][16];
    const int nkb = J.kp >> 4;
    int b = blockIdx.x, o = 0;
    while (o < 2 && b >= sel_groups(J.panels[o]) * nkb) b -= sel_groups(J.panels[o++]) * nkb;
    const int grp = b / nkb, kb = b % nkb;
    const int t = threadIdx.x;
    const int p0 = grp * kSelGroup, np = min(kSelGroup, J.panels[o] - p0);
    const uint16_t* X = (const uint16_t*)J.X[o];
    // the halves' swap depends on bits 2 and 3 of the point index only: the
    // same for this thread's point in every panel
    const int swz = row_swizzle(t);
    uint4 h[kSelGroup][2];
    float inv[kSelGroup];
#pragma unroll
    for (int q = 0; q < kSelGroup; ++q) {
        const int pn = p0 + min(q, np - 1);   // past the group's end: reread its last panel, dropped below
        const uint4* src = (const uint4*)(X + (((int64_t)pn * nkb + kb) * 128 + t) * 16);
        h[q][0] = src[0];
        h[q][1] = src[1];
        inv[q] = J.s[o] ? 1.0f / J.s[o][(int64_t)pn * 128 + t] : 1.0f;   // power of two: exact
    }
    float acc[16];   // in stored order
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
#pragma unroll
    for (int q = 0; q < kSelGroup; ++q) {
        if (q >= np) break;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t w = (&h[q][e >> 3].x)[(e & 7) >> 1];
            const uint16_t bits = (e & 1) ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xffff);
            float v;
            if constexpr (P == P_SPLIT16) v = (float)__builtin_bit_cast(_Float16, bits);
            else v = __uint_as_float((uint32_t)bits << 16);
            v *= inv[q];
            acc[e] += v * v;
        }
    }
    // stored position e holds row 16 kb + (e ^ 8 swz)
#pragma unroll
    for (int e = 0; e < 16; ++e) sq[t][e ^ (swz << 3)] = acc[e];
    __syncthreads();
    {
        const int k = t & 15, q = t >> 4;
        float a = 0.0f;
#pragma unroll
        for (int c = 0; c < 16; ++c) a += sq[q * 16 + c][k];
        part[q][k] = a;
    }
    __syncthreads();
    if (t < 16) {
        float a = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) a += part[q][t];
        J.part[o][(int64_t)grp * J.kp + kb * 16 + t] = a;
    }
}

// One workgroup: sums the groups' energies per row (FP64), scores the row
// pairs, ranks them, and writes the split count and the K-block order.  All
// pairs or none selected keep the natural order (then the contraction is
// the full split, or the high plane alone, bit for bit).
__global__ __launch_bounds__(1024) void row_select_kernel(SelJob J) {
    __shared__ double E[3][kMaxSelBlocks * 16];
    __shared__ double score[kMaxSelBlocks / 2];
    __shared__ int sorted[kMaxSelBlocks / 2];
    const int t = threadIdx.x;
    const int kp = J.kp, np = kp / 32;
    for (int o = 0; o < 3; ++o) {
        const int ng = sel_groups(J.panels[o]);
        for (int k = t; k < kp; k += 1024) {
            // independent partial sums, so that the loads overlap
            double a[4] = {0.0, 0.0, 0.0, 0.0};
            int g = 0;
            for (; g + 4 <= ng; g += 4)
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] += (double)J.part[o][(int64_t)(g + q) * kp + k];
            for (; g < ng; ++g) a[0] += (double)J.part[o][(int64_t)g * kp + k];
            E[o][k] = (a[0] + a[1]) + (a[2] + a[3]);
        }
    }
    __syncthreads();
    // a homocorrelation passes its A plane once (no panels for operand 1)
    const int o1 = J.panels[1] ? 1 : 0;
    if (t < np) {
        double a = 0.0;
        for (int k = 32 * t; k < 32 * t + 32; ++k) a += E[0][k] * (E[o1][k] + E[2][k]);
        score[t] = a;
    }
    __syncthreads();
    if (t < np) {
        int r = 0;
        for (int q = 0; q < np; ++q)
            r += (score[q] > score[t] || (score[q] == score[t] && q < t)) ? 1 : 0;
        sorted[r] = t;
    }
    __syncthreads();
    if (t == 0) {
        double total = 0.0;
        for (int r = 0; r < np; ++r) total += score[sorted[r]];
        // fewest leading pairs whose complement holds at most fmax of the total
        int c = 0;
        double tail = total;
        while (c < np && tail > J.fmax * total) tail -= score[sorted[c++]];
        J.sel[0] = 2 * c;
        const bool natural = c == 0 || c == np;
        for (int r = 0; r < np; ++r) {
            const int q = natural ? r : sorted[r];
            J.sel[1 + 2 * r] = 2 * q;
            J.sel[2 + 2 * r] = 2 * q + 1;
        }
    }
}

hipError_t launch_row_select(const SelJob& J, hipStream_t s) {
    const int blocks = (sel_groups(J.panels[0]) + sel_groups(J.panels[1]) + sel_groups(J.panels[2])) * (J.kp >> 4);
    if (J.prec == P_SPLIT16) hipLaunchKernelGGL(row_energy_kernel<P_SPLIT16>, dim3(blocks), dim3(128), 0, s, J);
    else hipLaunchKernelGGL(row_energy_kernel<P_SPLIT>, dim3(blocks), dim3(128), 0, s, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_select_kernel, dim3(1), dim3(1024), 0, s, J);
    return hipGetLastError();
}

// =========================================================================
// Interpolation onto the equidistant perturbation grid (FP64)
// =========================================================================
// Workgroup: 64 spectral points x 64 output rows; thread (c, s) owns output
// rows s, s+4, ... of column c.  The weights of the block's rows are staged
// through LDS in chunks of 64 input rows (read by a whole wave at once, a
// broadcast); only the block's nonzero input rows are visited.
__device__ inline double interp_load(const InterpJob& J, int64_t i, int64_t col) {
    return J.in_f64 ? ((const double*)J.y)[i * J.ld + col] : (double)((const float*)J.y)[i * J.ld + col];
}

__global__ __launch_bounds__(256) void interp_kernel(InterpJob J) {
    __shared__ double Wl[kInterpRows][64 + 1];
    const int tid = threadIdx.x, cl = tid & 63, rs = tid >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + cl;
    const int64_t k0 = (int64_t)blockIdx.y * kInterpRows;
    const int lo = J.range[2 * blockIdx.y], hi = J.range[2 * blockIdx.y + 1];
    double acc[kInterpRows / 4];
#pragma unroll
    for (int q = 0; q < kInterpRows / 4; ++q) acc[q] = 0.0;
    for (int i0 = lo; i0 < hi; i0 += 64) {
        __syncthreads();   // previous chunk's readers are done
        for (int e = tid; e < kInterpRows * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int64_t k = k0 + r, i = i0 + c;
            Wl[r][c] = (k < J.N && i < hi) ? J.W[k * J.m_in + i] : 0.0;
        }
        __syncthreads();
        const int ie = hi - i0 < 64 ? hi - i0 : 64;
        if (col < J.n) {
            for (int ii = 0; ii < ie; ++ii) {
                const double y = interp_load(J, i0 + ii, col);
#pragma unroll
                for (int q = 0; q < kInterpRows / 4; ++q) acc[q] += Wl[rs + 4 * q][ii] * y;
            }
        }
    }
    if (col < J.n) {
#pragma unroll
        for (int q = 0; q < kInterpRows / 4; ++q) {
            const int64_t k = k0 + rs + 4 * q;
            if (k < J.N) J.out[k * J.ld_out + col] = acc[q];
        }
    }
}

// =========================================================================
// Host launchers
// =========================================================================
hipError_t launch_tables_qn(const TableSrcInline& src, int blocks, int64_t max_m, hipStream_t s) {
    hipLaunchKernelGGL(tables_qn_kernel<TableSrcInline>, dim3(blocks), dim3(256), (size_t)(16 * max_m), s, src);
    return hipGetLastError();
}
hipError_t launch_tables_qn(const TableSrcArray& src, int blocks, int64_t max_m, hipStream_t s) {
    hipLaunchKernelGGL(tables_qn_kernel<TableSrcArray>, dim3(blocks), dim3(256), (size_t)(16 * max_m), s, src);
    return hipGetLastError();
}
hipError_t launch_interp(const InterpJob& J, hipStream_t s) {
    const dim3 grid((unsigned)((J.n + 63) / 64), (unsigned)((J.N + kInterpRows - 1) / kInterpRows));
    hipLaunchKernelGGL(interp_kernel, grid, dim3(256), 0, s, J);
    return hipGetLastError();
}

hipError_t launch_tables(const TableSrcInline& src, int blocks, int64_t max_m, hipStream_t s) {
    hipLaunchKernelGGL(tables_kernel<TableSrcInline>, dim3(blocks), dim3(256), (size_t)(32 * max_m), s, src);
    return hipGetLastError();
}
hipError_t launch_tables(const TableSrcArray& src, int blocks, int64_t max_m, hipStream_t s) {
    hipLaunchKernelGGL(tables_kernel<TableSrcArray>, dim3(blocks), dim3(256), (size_t)(32 * max_m), s, src);
    return hipGetLastError();
}
hipError_t launch_prep(const TableSrcInline& ts, int nt, int nq, int64_t m, const PrepSrcInline& ps, int nc,
                       hipStream_t s) {
    hipLaunchKernelGGL(prep_kernel, dim3(nt + nq + nc), dim3(256), (size_t)(32 * m), s, ts, nt, nq, ps);
    return hipGetLastError();
}
hipError_t launch_center(const PrepSrcInline& src, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(center_kernel<PrepSrcInline>, dim3(blocks), dim3(256), 0, s, src);
    return hipGetLastError();
}
hipError_t launch_center(const PrepSrcArray& src, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(center_kernel<PrepSrcArray>, dim3(blocks), dim3(256), 0, s, src);
    return hipGetLastError();
}

template <class Src>
static hipError_t launch_transform_t(int prec, const Src& src, int blocks, hipStream_t s) {
    switch (prec) {
    case P_F64: hipLaunchKernelGGL((transform_kernel<P_F64, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_F32: hipLaunchKernelGGL((transform32_kernel<P_F32, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_SPLIT: hipLaunchKernelGGL((transform32_kernel<P_SPLIT, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_BF16: hipLaunchKernelGGL((transform32_kernel<P_BF16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_F16: hipLaunchKernelGGL((transform32_kernel<P_F16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_SPLIT16: hipLaunchKernelGGL((transform32_kernel<P_SPLIT16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_FP8: hipLaunchKernelGGL((transform32_kernel<P_FP8, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <class Src>
static hipError_t launch_center_transform_t(int prec, const Src& src, int blocks, hipStream_t s) {
    switch (prec) {
    case P_F32: hipLaunchKernelGGL((center_transform32_kernel<P_F32, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_SPLIT: hipLaunchKernelGGL((center_transform32_kernel<P_SPLIT, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_BF16: hipLaunchKernelGGL((center_transform32_kernel<P_BF16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_F16: hipLaunchKernelGGL((center_transform32_kernel<P_F16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_SPLIT16: hipLaunchKernelGGL((center_transform32_kernel<P_SPLIT16, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    case P_FP8: hipLaunchKernelGGL((center_transform32_kernel<P_FP8, Src>), dim3(blocks), dim3(256), 0, s, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t launch_center_transform(int prec, const PrepSrcInline& src, int blocks, hipStream_t s) {
    return launch_center_transform_t(prec, src, blocks, s);
}
hipError_t launch_center_transform(int prec, const PrepSrcArray& src, int blocks, hipStream_t s) {
    return launch_center_transform_t(prec, src, blocks, s);
}
hipError_t launch_transform(int prec, const PrepSrcInline& src, int blocks, hipStream_t s) {
    return launch_transform_t(prec, src, blocks, s);
}

hipError_t launch_fft_tables(const TableSrcInline& src, int64_t m, hipStream_t s) {
    hipLaunchKernelGGL(fft_tables_kernel<TableSrcInline>, dim3((unsigned)(2 * m)), dim3(256), 0, s, src);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_fft_p(int log2l, const PrepSrcInline& src, int blocks, hipStream_t s) {
    switch (log2l) {
    case 8: hipLaunchKernelGGL((fft_transform_kernel<P, 8, PrepSrcInline>), dim3(blocks), dim3(256), 0, s, src); break;
    case 9: hipLaunchKernelGGL((fft_transform_kernel<P, 9, PrepSrcInline>), dim3(blocks), dim3(256), 0, s, src); break;
    case 10: hipLaunchKernelGGL((fft_transform_kernel<P, 10, PrepSrcInline>), dim3(blocks), dim3(256), 0, s, src); break;
    case 11: hipLaunchKernelGGL((fft_transform_kernel<P, 11, PrepSrcInline>), dim3(blocks), dim3(256), 0, s, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_transform(int prec, int log2l, const PrepSrcInline& src, int blocks, hipStream_t s) {
    switch (prec) {
    case P_F64: return launch_fft_p<P_F64>(log2l, src, blocks, s);
    case P_F32: return launch_fft_p<P_F32>(log2l, src, blocks, s);
    case P_SPLIT: return launch_fft_p<P_SPLIT>(log2l, src, blocks, s);
    case P_BF16: return launch_fft_p<P_BF16>(log2l, src, blocks, s);
    case P_F16: return launch_fft_p<P_F16>(log2l, src, blocks, s);
    case P_SPLIT16: return launch_fft_p<P_SPLIT16>(log2l, src, blocks, s);
    case P_FP8: return launch_fft_p<P_FP8>(log2l, src, blocks, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_transform(int prec, const PrepSrcArray& src, int blocks, hipStream_t s) {
    return launch_transform_t(prec, src, blocks, s);
}

#define CORR_CASES(X) X(P_F64, 2, 2) X(P_F64, 4, 2) X(P_F32, 4, 4) X(P_FP8, 4, 4) X(P_F32, 2, 2) X(P_FP8, 2, 2)
#define CORR2_CASES(X) X(P_SPLIT) X(P_BF16) X(P_F16) X(P_SPLIT16)

hipError_t launch_corr(int prec, int fm, int fn, const CorrJob& C, int64_t blocks, hipStream_t s) {
    // row-selective split: the kernels that read the K-block order
    if (C.kb_sel && (prec == P_SPLIT || prec == P_SPLIT16) && (fm == 8 || fm == 4) && fn == 4) {
        if (prec == P_SPLIT) {
            if (fm == 8) hipLaunchKernelGGL((corr2_kernel<P_SPLIT, 256, true>), dim3((unsigned)blocks), dim3(512), 0, s, C);
            else hipLaunchKernelGGL((corr2_kernel<P_SPLIT, 128, true>), dim3((unsigned)blocks), dim3(256), 0, s, C);
        } else {
            if (fm == 8) hipLaunchKernelGGL((corr2_kernel<P_SPLIT16, 256, true>), dim3((unsigned)blocks), dim3(512), 0, s, C);
            else hipLaunchKernelGGL((corr2_kernel<P_SPLIT16, 128, true>), dim3((unsigned)blocks), dim3(256), 0, s, C);
        }
        return hipGetLastError();
    }
#define Y(PP)                                                                                 \
    if (prec == PP && (fm == 8 || fm == 4) && fn == 4) {                                      \
        if (fm == 8) hipLaunchKernelGGL((corr2_kernel<PP, 256>), dim3((unsigned)blocks), dim3(512), 0, s, C); \
        else hipLaunchKernelGGL((corr2_kernel<PP, 128>), dim3((unsigned)blocks), dim3(256), 0, s, C); \
        return hipGetLastError();                                                             \
    }
    CORR2_CASES(Y)
#undef Y
#define X(PP, A, B)                                                                          \
    if (prec == PP && fm == A && fn == B) {                                                  \
        hipLaunchKernelGGL((corr_kernel<PP, A, B>), dim3((unsigned)blocks), dim3(256),         \
                           corr_lds_bytes(A, B, C.out_f64), s, C);                           \
        return hipGetLastError();                                                            \
    }
    CORR_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_corr_persistent(int prec, int fm, int fn, bool out_f64, const CorrJob* jobs,
                                  const int64_t* tile_start, int count, int64_t total,
                                  int* counter, int blocks, hipStream_t s) {
#define Y(PP)                                                                                 \
    if (prec == PP && (fm == 8 || fm == 4) && fn == 4) {                                      \
        if (fm == 8)                                                                          \
            hipLaunchKernelGGL((corr2_persistent_kernel<PP, 256>), dim3(blocks), dim3(512), 0, s, jobs, \
                               tile_start, count, total, counter);                            \
        else                                                                                  \
            hipLaunchKernelGGL((corr2_persistent_kernel<PP, 128>), dim3(blocks), dim3(256), 0, s, jobs, \
                               tile_start, count, total, counter);                            \
        return hipGetLastError();                                                             \
    }
    CORR2_CASES(Y)
#undef Y
#define X(PP, A, B)                                                                         \
    if (prec == PP && fm == A && fn == B) {                                                 \
        hipLaunchKernelGGL((corr_persistent_kernel<PP, A, B>), dim3(blocks), dim3(256),        \
                           corr_lds_bytes(A, B, out_f64), s, jobs, tile_start, count, total, counter); \
        return hipGetLastError();                                                           \
    }
    CORR_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

int corr_variant_supported(int prec, int fm, int fn) {
#define Y(PP) if (prec == PP && (fm == 8 || fm == 4) && fn == 4) return 1;
    CORR2_CASES(Y)
#undef Y
#define X(PP, A, B) if (prec == PP && fm == A && fn == B) return 1;
    CORR_CASES(X)
#undef X
    return 0;
}

int persistent_blocks_per_cu(int prec, int fm, int fn, bool out_f64) {
    int n = 0;
#define Y(PP)                                                                             \
    if (prec == PP && (fm == 8 || fm == 4) && fn == 4) {                                  \
        const hipError_t e = fm == 8                                                      \
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr2_persistent_kernel<PP, 256>, 512, 0) \
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr2_persistent_kernel<PP, 128>, 256, 0); \
        if (e != hipSuccess) n = 1;                                                       \
        return n > 0 ? n : 1;                                                             \
    }
    CORR2_CASES(Y)
#undef Y
#define X(PP, A, B)                                                                      \
    if (prec == PP && fm == A && fn == B) {                                              \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr_persistent_kernel<PP, A, B>, 256, \
                                                         corr_lds_bytes(A, B, out_f64)) != hipSuccess) \
            n = 1;                                                                       \
        return n > 0 ? n : 1;                                                            \
    }
    CORR_CASES(X)
#undef X
    return 1;
}

}  // namespace corr2d
