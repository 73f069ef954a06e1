// corr2d_internal.h -- descriptors shared by the host plan code and the HIP
// kernels of the correlation library.  Plain structs only; no HIP types.
#pragma once
#include <stdint.h>

namespace corr2d {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_SPLIT = 2, P_BF16 = 3, P_F16 = 4, P_FP8 = 5, P_SPLIT16 = 6 };
enum Basis : int { B_FOURIER = 0, B_TIME = 1 };
enum Hilbert : int { H_NODA = 0, H_CIRCULAR = 1, H_R_COMPAT = 2 };
enum Layout : int { L_FULL = 0, L_UPPER = 1, L_UPPER_ALIGNED = 2 };

// 16-bit formats use the LDS-staged contraction kernel and the K-blocked
// operand layout (see blocked_index); the others the register-direct kernel
// and the row layout [i][kp].
__host__ __device__ constexpr bool blocked_layout(int prec) {
    return prec == P_SPLIT || prec == P_BF16 || prec == P_F16 || prec == P_SPLIT16;
}

// Contraction length granularity per precision (the LDS-staged kernel of
// the 16-bit formats takes its K blocks of 16 in pairs).
__host__ __device__ constexpr int k_align(int prec) {
    return prec == P_FP8 ? 64 : blocked_layout(prec) ? 32 : 16;
}

// Panel-blocked operand layout of the 16-bit formats.  Rows are grouped in
// panels of 128; a panel holds its K blocks of 16 elements one after another,
// each block as 128 rows x 32 bytes (the two 8-element halves of the block,
// swapped for rows with ((i >> 2) ^ (i >> 3)) & 1 set).  A contraction stage
// (one K block of one panel) is then a contiguous 4 KB run that the
// contraction kernel copies linearly into LDS, where the swap spreads the
// 32x32 MFMA fragment reads of 16 consecutive rows over all LDS banks; and
// the whole K range of a panel is one contiguous 64 KB run, so the K blocks
// of a tile never alias to the same L2 sets.
__host__ __device__ constexpr int row_swizzle(int64_t i) { return (int)(((i >> 2) ^ (i >> 3)) & 1); }
__host__ __device__ constexpr int64_t blocked_index(int64_t i, int64_t k, int64_t kp) {
    return (((i >> 7) * (kp >> 4) + (k >> 4)) * 128 + (i & 127)) * 16 +
           ((((k >> 3) & 1) ^ row_swizzle(i)) << 3) + (k & 7);
}
__host__ __device__ constexpr int elem_bytes(int prec) {
    return prec == P_F64 ? 8 : prec == P_F32 ? 4 : prec == P_FP8 ? 1 : 2;
}
__host__ __device__ constexpr int planes(int prec) { return prec == P_SPLIT || prec == P_SPLIT16 ? 2 : 1; }

constexpr int kTransformK = 16;   // inner-dimension granularity of the transform GEMM
constexpr int kTransformTile = 64;
constexpr int kNPad = 128;        // spectral points are padded to this multiple
constexpr int kCenterCols = 32;   // columns per workgroup of the centring kernel

// Transform table of one perturbation length: rows [0, kp) are the operand
// transform T1, rows [kp, 2kp) the asynchronous operand transform T2, rows up
// to rows_pad are zero.  Row-major, rows_pad x kt, double (FP64 transform) or
// float.
struct TableJob {
    int64_t m;
    int32_t kp, kt, rows_pad;
    int32_t basis, hilbert;
    int32_t f64;
    void* table;
};

// Preparation of one data set: centring, transform and packing.
struct PrepJob {
    const void* y;        // m x ld input spectra (device)
    const double* ref;    // reference spectrum or nullptr (mean)
    int64_t ld;
    int64_t m, n, n_pad;
    int32_t kp, kt, rows_pad;
    int32_t in_f64;       // 1: y is double, 0: float
    int32_t t_f64;        // 1: transform in FP64 (tables/yt double)
    int32_t prec;
    int32_t need_b;       // produce the asynchronous operand B
    int32_t scale;        // per-band power-of-two scales
    float qhalf;          // half of the format's largest finite value
    float pad0;
    double boundA, boundB; // max|operand column| <= bound * ||centred column||_2
    void* yt;             // n_pad x kt centred spectra, transposed (workspace)
    const void* table;    // transform table (workspace)
    float* sA;            // n_pad scales of operand A
    float* sB;            // n_pad scales of operand B
    void* A0; void* A1;   // operand A planes, n_pad x kp (A1: split low plane)
    void* B0; void* B1;   // operand B planes
    double alpha;         // result scaling exponent (0: none): columns x sigma^-alpha
    int32_t hilbert;      // Hilbert and Basis (the radix FFT transform builds
    int32_t basis;        // the operands from them, without a table)
    double* ref_out;      // n doubles (workspace): the reference spectrum the
                          // centring subtracted (the mean, or a copy of ref)
};

// Resampling of one data set onto the equidistant perturbation grid: out =
// W y (FP64), W N x m_in; range[2b], range[2b+1] bound the nonzero input rows
// of output rows [b kInterpRows, (b+1) kInterpRows).
constexpr int kInterpRows = 64;
struct InterpJob {
    const void* y;        // m_in x ld input spectra (device)
    int64_t ld, n, m_in, N;
    int32_t in_f64;       // 1: y is double, 0: float
    int32_t pad0;
    const double* W;      // N x m_in (workspace)
    const int32_t* range; // (workspace)
    double* out;          // N x ld_out (workspace)
    int64_t ld_out;
};

// One correlation contraction (a homocorrelation or a heterocorrelation).
// Outputs of a call up to this size (both planes) are written with
// system-scope stores by the direct epilogue, larger ones non-temporally:
// measured on the 16-bit kernel, system-scope stores are 3-10 % faster while
// the outputs fit the 256 MB memory-side cache, and 10-23 % slower beyond.
constexpr int64_t kNearStoreBytes = int64_t(192) << 20;

// Row selection of the split formats (Fourier basis): the energy of every
// packed Fourier row k of each operand, E_X[k] = sum_nu (X[k][nu] / s_nu)^2
// from the high plane, then the K-block order of the contraction.  Operands:
// 0 the left A, 1 the right A, 2 the right B (a homocorrelation gives
// operand 1 no panels: its right A is operand 0).  Row pairs of K blocks (32 rows) are ranked by
// sum_k E_0[k] (E_1[k] + E_2[k]), the energy of the hi*hi rounding errors of
// their products, and the fewest leading pairs whose complement holds at
// most fmax of that energy keep the low plane.
constexpr int kMaxSelBlocks = 64;   // K blocks a selection orders (kp <= 1024)
constexpr int kSelGroup = 8;        // panels of 128 points per energy workgroup
__host__ __device__ constexpr int sel_groups(int panels) { return (panels + kSelGroup - 1) / kSelGroup; }
struct SelJob {
    const void* X[3];      // high planes (panel-blocked)
    const float* s[3];     // per-band scales (nullptr: unscaled)
    float* part[3];        // row energies per group of kSelGroup panels:
                           // sel_groups(panels_o) x kp floats each
    int32_t panels[3];     // column panels of 128 per operand
    int32_t kp;
    int32_t prec;
    double fmax;           // fraction of the error energy left to hi*hi
    int32_t* sel;          // [0] split K blocks, then the kp/16 K-block order
};

struct CorrJob {
    const void* L0; const void* L1;   // left operand planes (set 1, A)
    const void* RA0; const void* RA1; // right synchronous operand (set 2, A)
    const void* RB0; const void* RB1; // right asynchronous operand (set 2, B)
    const float* sL; const float* sRA; const float* sRB;
    void* phi; void* psi;
    int64_t n1, n2;     // true sizes
    int64_t ld_out;     // FULL row stride
    int32_t kp;
    int32_t tiles_i, tiles_j;   // tile grid
    int32_t homo;       // 1: upper-triangle tiles only, mirror or pack
    int32_t layout;     // Layout
    int32_t out_f64;
    int32_t group;      // column tiles per L2 group
    int32_t scaled;     // operands carry per-band power-of-two scales
    int32_t ratio;      // row tile height / column tile width (homo tile order)
    int32_t store_near; // 1: the call's outputs fit the memory-side cache (see
                        // kNearStoreBytes): direct stores at system scope
    int64_t ntiles;
    double c;           // FP64 normalization of the contraction
    // Row-selective split (split formats, nullptr otherwise): [0] the number
    // of K blocks (an even count, leading the order) that carry the low
    // plane, then the order of the kp/16 K blocks (at most 64), written by
    // the selection kernel of the same call.
    const int32_t* kb_sel;
};

}  // namespace corr2d
