/*
 * corr2d.h -- C ABI of the MI355X (gfx950) generalized two-dimensional
 * correlation library.
 *
 * What it computes (Geitner et al., "corr2D", arXiv 1808.00685, Sec. 2):
 * given m spectra of n points, taken at m equidistant perturbation steps,
 *   1. dynamic spectra  y~(nu, t) = y(nu, t) - r(nu), where r is the
 *      perturbation mean spectrum (Eqs. (dynspec), (ref)) or a reference
 *      spectrum the caller supplies (Sec. 4.2);
 *   2. a Fourier transform along the perturbation axis (Eq. (disFT)), kept as
 *      the Hermitian half spectrum of a real signal (Eq. (symmeFT), Sec. 4.2);
 *   3. the complex correlation  Phi + i Psi  between every pair of spectral
 *      points as a contraction over the Fourier frequencies of F1 conj(F2),
 *      scaled by the normalization (Eq. (disint2d), Sec. 4.2 "Norm").
 * Phi (synchronous) is symmetric and Psi (asynchronous) antisymmetric for a
 * homocorrelation (one data set with itself, Sec. 2 end and Sec. 3).
 *
 * The asynchronous kernel.  With the default CORR2D_HILBERT_NODA, Psi equals
 * Noda's direct formula Y1^T N Y2 / (m-1) with the Hilbert-Noda matrix N
 * (Eqs. (disHT), (HilbNoda), (disHTasyn)); it is evaluated as a Fourier
 * contraction of F1 against the transform of N Y2, which is exact.
 * CORR2D_HILBERT_CIRCULAR takes the imaginary part of the m-point half
 * spectrum product literally (the discrete Fourier route of Eq. (disint2d));
 * for finite m it differs from Noda's kernel.  Phi is the same in both.
 * CORR2D_HILBERT_R_COMPAT evaluates the m-point route over the bin list of
 * the package's R code (Sec. 4.2), which weighs the top bin differently
 * (Phi differs too); with CORR2D_NORM_PAPER it reproduces that code.
 *
 * Normalization.  The factor cF multiplies the Hermitian-weighted Fourier sum
 * sum_w weight(w) F1(w) conj(F2(w)) (weight 1 for DC and Nyquist, 2 else):
 *   CORR2D_NORM_NODA   cF = 1/(m (m-1))   -> Phi = Y1^T Y2/(m-1)   (default)
 *   CORR2D_NORM_PAPER  cF = 1/(pi (m-1))  -> the paper's default "Norm";
 *                                            exactly m/pi times NODA
 *   CORR2D_NORM_CUSTOM cF = desc.norm_value
 *
 * Memory.  Every data pointer passed to a compute call is device memory owned
 * by the caller (for example a torch tensor).  Input spectra are row-major
 * m x ld (row t = the spectrum at perturbation step t, each spectrum
 * contiguous, the paper's input matrix of Sec. 3).  Full outputs are
 * row-major n1 x ld_out.  UPPER_PACKED (homocorrelation only) stores row i's
 * entries j = i..n-1 contiguously at offset i*n - i*(i-1)/2 + (j - i).
 * UPPER_ALIGNED (homocorrelation only) stores the same entries with every row
 * starting on a 32-element boundary (128 bytes of FP32): row i covers the
 * columns c(i) = 32*floor(i/32) .. N32-1, N32 = n rounded up to a multiple of
 * 32, so element (i, j), j >= i, sits at corr2d_upper_aligned_index(i, j, n)
 * below.  The slots of columns c(i)..i-1 and n..N32-1 are padding that the
 * library never writes; one plane holds corr2d_upper_aligned_elements(n)
 * elements (n (n+1)/2 plus at most 62 n).  Stores of whole cache lines make
 * this layout faster to write than UPPER_PACKED, whose rows start mid-line.
 * A plan owns host memory only and can be created without a GPU.
 *
 * Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 * void*, NULL = the default stream).  CORR2D_OK means the work was enqueued;
 * results are valid after the stream is synchronized.  Argument errors are
 * reported before any device work.  No C++ exception crosses this boundary.
 * NaN or Inf in the inputs propagate; the hot path does not inspect values.
 * A plan may be used from several streams at once provided every concurrent
 * call has its own workspace.
 */
#ifndef CORR2D_H
#define CORR2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum corr2d_status {
    CORR2D_OK = 0,
    CORR2D_EINVAL = 1,      /* invalid argument (sizes, pointers, enums)       */
    CORR2D_EWORKSPACE = 2,  /* workspace missing, misaligned or too small      */
    CORR2D_EUNSUPPORTED = 3,/* valid but unsupported combination               */
    CORR2D_EDEVICE = 4,     /* a HIP runtime call failed (see corr2d_last_error)*/
    CORR2D_ENOMEM = 5       /* host allocation failed                          */
} corr2d_status;

/* Arithmetic of the contraction (step 3).  Mean subtraction and the final
 * normalization are always FP64; the transform (step 2) is FP64 for
 * CORR2D_PREC_F64 and FP32 otherwise.  Reduced precisions accumulate in FP32. */
typedef enum corr2d_prec {
    CORR2D_PREC_F64 = 0,        /* FP64 MFMA                                    */
    CORR2D_PREC_F32 = 1,        /* FP32 MFMA                                    */
    CORR2D_PREC_SPLIT_BF16 = 2, /* x = hi + lo (both BF16); hi*hi+hi*lo+lo*hi   */
    CORR2D_PREC_BF16 = 3,       /* plain BF16                                   */
    CORR2D_PREC_F16 = 4,        /* FP16, per-band scaling on by default          */
    CORR2D_PREC_FP8_E4M3 = 5,   /* OCP FP8 e4m3, per-band scaling required      */
    CORR2D_PREC_SPLIT_F16 = 6   /* x = hi + lo (both FP16) after the per-band
                                   power-of-two scale (required); hi*hi+hi*lo+
                                   lo*hi: 11-bit halves, per-product error
                                   about 2^-22 against split BF16's 2^-16     */
} corr2d_prec;

/* Basis of the contraction.  FOURIER contracts the real-packed Hermitian half
 * spectrum (the paper's Fourier route).  TIME contracts the dynamic spectra
 * directly (the paper's Hilbert-transform route).  Both give the same Phi and
 * Psi up to rounding; they differ in how rounding errors of reduced precisions
 * accumulate.                                                                 */
typedef enum corr2d_basis {
    CORR2D_BASIS_FOURIER = 0,
    CORR2D_BASIS_TIME = 1,
    CORR2D_BASIS_AUTO = 2   /* the default: TIME (the operands' rounding
                               errors then spread over all m products instead
                               of concentrating in the few Fourier rows that
                               carry the bands: 2-9x smaller errors in the
                               reduced formats, the same cost), FOURIER with
                               CORR2D_HILBERT_R_COMPAT or
                               CORR2D_FLAG_SPLIT_ROWS, which need it        */
} corr2d_basis;
typedef enum corr2d_hilbert {
    CORR2D_HILBERT_NODA = 0,      /* Noda's matrix, Eq. (HilbNoda)                   */
    CORR2D_HILBERT_CIRCULAR = 1,  /* m-point route, Hermitian-complete half spectrum */
    CORR2D_HILBERT_R_COMPAT = 2   /* m-point route with the bin list of the package's
                                     R code (Sec. 4.2): bins floor(j/2), j = 1..m-1
                                     (DC once, top bin once for odd m, no Nyquist
                                     bin for even m); Fourier basis only            */
} corr2d_hilbert;
typedef enum corr2d_norm { CORR2D_NORM_NODA = 0, CORR2D_NORM_PAPER = 1, CORR2D_NORM_CUSTOM = 2 } corr2d_norm;
typedef enum corr2d_layout {
    CORR2D_LAYOUT_FULL = 0,
    CORR2D_LAYOUT_UPPER_PACKED = 1,
    CORR2D_LAYOUT_UPPER_ALIGNED = 2
} corr2d_layout;

/* Offset of element (i, j), 0 <= i <= j < n, in the UPPER_ALIGNED layout:
 * with i = 32 q + r, row i starts at i*N32 - 32 (16 q (q-1) + r q), the sum
 * of the lengths N32 - 32 floor(k/32) of the rows k < i.                    */
static inline int64_t corr2d_upper_aligned_index(int64_t i, int64_t j, int64_t n) {
    const int64_t n32 = (n + 31) / 32 * 32, q = i / 32, r = i % 32;
    return i * n32 - 32 * (16 * q * (q - 1) + r * q) + (j - 32 * q);
}
/* Elements of one UPPER_ALIGNED output plane of an n x n correlation.      */
static inline int64_t corr2d_upper_aligned_elements(int64_t n) {
    return corr2d_upper_aligned_index(n, 32 * (n / 32), n);
}
typedef enum corr2d_dtype { CORR2D_DTYPE_F64 = 0, CORR2D_DTYPE_F32 = 1 } corr2d_dtype;

/* desc.flags */
#define CORR2D_FLAG_PER_BAND_SCALE 0x1u  /* power-of-two scale per spectral point */
#define CORR2D_FLAG_NO_PER_BAND_SCALE 0x2u /* force scaling off (F16 only)          */
#define CORR2D_FLAG_SEQUENTIAL 0x4u      /* batched: one launch chain per data set */
#define CORR2D_FLAG_NO_GRAPH 0x8u        /* batched: launch directly, no hipGraph  */
/* Row-selective split (split formats, Fourier basis, m <= 1024, single and
 * heterocorrelation plans): the low plane enters only the products of the
 * packed Fourier rows that carry most of the energy (Eq. (symmeFT): a band
 * spectrum's dynamic spectra concentrate in the low frequencies).  Each
 * call measures the energy of every row of its operands, ranks the pairs
 * of 16-row K blocks by the energy of their hi*hi rounding errors, and
 * keeps the low plane for the fewest leading pairs whose complement holds
 * at most the fraction of that energy which the target desc.split_tol
 * allows (the modelled relative error of Phi from the rows left to hi*hi
 * is an eighth of the target).  The target bounds Phi's modelled error; Psi
 * follows it unless Psi itself cancels strongly.  The selection is written
 * to the workspace (plan info sel_offset).                                 */
#define CORR2D_FLAG_SPLIT_ROWS 0x20u
#define CORR2D_FLAG_TRANSFORM_MATMUL 0x10u /* perturbation-axis transform as the MFMA
                                           product with the table also where the
                                           radix FFT applies (power-of-two
                                           128 <= m <= 1024; Fourier basis, or
                                           time basis with Noda's kernel)      */

typedef struct corr2d_desc {
    int64_t m;          /* perturbation steps, >= 2 (Eq. (disFT): equidistant)   */
    int64_t n1;         /* spectral points of the first (or only) data set, >= 1 */
    int64_t n2;         /* spectral points of the second set; 0 = homocorrelation */
    int64_t ld_in1;     /* row stride of y1 in elements; 0 = n1                  */
    int64_t ld_in2;     /* row stride of y2 in elements; 0 = n2                  */
    int64_t ld_out;     /* row stride of FULL outputs in elements; 0 = columns   */
    int32_t in_dtype;   /* corr2d_dtype of y1, y2 (references are always FP64)  */
    int32_t out_dtype;  /* corr2d_dtype of phi, psi                             */
    int32_t prec;       /* corr2d_prec                                           */
    int32_t basis;      /* corr2d_basis                                          */
    int32_t hilbert;    /* corr2d_hilbert                                        */
    int32_t norm_mode;  /* corr2d_norm                                           */
    double norm_value;  /* cF for CORR2D_NORM_CUSTOM                             */
    int32_t out_layout; /* corr2d_layout                                         */
    uint32_t flags;     /* CORR2D_FLAG_*                                         */
    int32_t tile;       /* 0 = automatic (tuned table); 1 = 64 x 64 output tiles
                           (FP64, FP32, FP8); 2 = 128 x 128 (FP32, FP8),
                           128 x 64 (FP64) or 256 x 128 (split-BF16, BF16,
                           FP16); 3 = 128 x 128 (split-BF16, BF16, FP16)       */
    int32_t reserved;
    double scale_alpha; /* exponent alpha of the result scaling: Phi and Psi
                           divided by (sigma_1 sigma_2)^alpha, Sec. 2 Eqs.
                           (stdev), (scalesyn), (scaleasyn); 0 = unscaled,
                           1 = Pearson, 0.5 = Pareto.  sigma per spectral
                           variable from the dynamic spectrum in use; a
                           variable with sigma = 0 stays unscaled.  Finite.     */
    /* Interpolation to equidistant perturbation values (Sec. 4.1).  With
     * interp != CORR2D_INTERP_NONE the input spectra have m_in rows taken at
     * the perturbation values t_in[0..m_in-1] (host memory, strictly
     * increasing, read when the plan is made); each spectral variable is
     * resampled on the m equidistant values t_in[0] + k (t_in[m_in-1] -
     * t_in[0]) / (m-1), in FP64, before the correlation.  Not for batched
     * plans.                                                                  */
    const double* t_in;
    int64_t m_in;
    int32_t interp;     /* corr2d_interp                                          */
    int32_t reserved2;
    double split_tol;   /* CORR2D_FLAG_SPLIT_ROWS: target relative error of the
                           result (finite, >= 0; 0 = 1e-5)                      */
} corr2d_desc;

/* Interpolation of Sec. 4.1: piecewise linear (R's approxfun), or the cubic
 * spline with the end conditions of Forsythe, Malcolm and Moler (the default
 * method of R's splinefun): end third derivatives equal those of the cubics
 * through the first and last four points; three points give the parabola
 * through them, two the line.                                                 */
typedef enum corr2d_interp {
    CORR2D_INTERP_NONE = 0,
    CORR2D_INTERP_LINEAR = 1,
    CORR2D_INTERP_SPLINE = 2
} corr2d_interp;

/* One data set of a batched homocorrelation.  Offsets are in elements from
 * the base pointers given to corr2d_batched.                                   */
typedef struct corr2d_item {
    int64_t m;          /* perturbation steps of this set, >= 2                   */
    int64_t n;          /* spectral points, >= 1                                  */
    int64_t in_offset;  /* y of this set starts at y_base + in_offset             */
    int64_t ld_in;      /* its row stride; 0 = n                                  */
    int64_t out_offset; /* phi/psi of this set start at base + out_offset         */
} corr2d_item;

typedef struct corr2d_plan_s* corr2d_plan_t;

/* Read-only facts about a plan (for logging and benchmarks).                  */
typedef struct corr2d_plan_info {
    int64_t k_pad;        /* contraction length after padding                     */
    int64_t n_pad;        /* spectral points after padding to the tile            */
    int64_t tiles;        /* output tiles one call computes                       */
    int32_t tile;         /* corr2d tile id in use                                */
    int32_t tile_m;       /* output tile rows                                     */
    int32_t tile_n;       /* output tile columns                                  */
    int32_t per_band_scale;
    double c;             /* final FP64 factor applied to the contraction         */
    size_t workspace_bytes;
    int64_t items;        /* batched plans: data sets                             */
    int64_t out_elements; /* batched plans: elements of phi (and of psi) written  */
    int32_t transform;    /* perturbation-axis transform: 0 = product with the DFT
                             table on MFMA, 1 = radix FFT in LDS                  */
    int32_t basis;        /* corr2d_basis in use (AUTO resolved)                  */
    /* Single and hetero plans: byte offsets in the workspace of the reference
     * spectra a call subtracts (Sec. 2 Eqs. (dynspec), (ref); the Ref1 and
     * Ref2 of the paper's result object, Sec. 3): n1 (n2) doubles, the
     * perturbation mean computed in FP64, or a copy of the caller's ref1
     * (ref2).  Written by every call, readable once it has completed, until
     * the workspace is used again.  Homocorrelation: ref2_offset equals
     * ref1_offset.  Batched plans: 0 (not reported).                         */
    size_t ref1_offset;
    size_t ref2_offset;
    /* CORR2D_FLAG_SPLIT_ROWS: byte offset in the workspace of the selection
     * record a call writes (readable once the call has completed): int32
     * count of the K blocks of 16 packed rows that carried the low plane,
     * then the order of the k_pad/16 K blocks, those first.  0 otherwise.  */
    size_t sel_offset;
} corr2d_plan_info;

/* Fill *d with defaults: FP64 input, FP32 output, SPLIT_BF16, AUTO basis, NODA
 * kernel and norm, FULL layout, automatic tile.  The caller sets m, n1, n2.  */
void corr2d_desc_init(corr2d_desc* d);

/* Validate d and build a plan in host memory.  No device call is made.
 * The descriptor carries the arguments of the paper's corr2d() call (Sec. 3,
 * Sec. 4.2): the data sets' sizes, the reference (Ref1/Ref2 at call time),
 * Norm (norm_mode), scaling (scale_alpha), Time/Int/N (interpolation,
 * Sec. 4.1), plus this library's choices of arithmetic and output layout.
 * A plan is immutable once made: the compute calls read it and never change
 * it (a batched plan's cached graph and job buffer are internal, guarded by
 * a lock).                                                                  
 * EINVAL: m < 2, n1 < 1, n2 < 0, a stride smaller than its row, an unknown
 * enum value, CUSTOM norm with a non-finite norm_value, UPPER_PACKED or
 * UPPER_ALIGNED for a heterocorrelation.  EUNSUPPORTED: FP8 with per-band scaling forced off.   */
corr2d_status corr2d_plan(corr2d_plan_t* out, const corr2d_desc* d);

/* Batched homocorrelation of count independent data sets (count >= 1):
 * corr2d(Mat1) of Sec. 3 applied to each set.  The paper measures that the
 * per-call setup dominates small problems (Sec. 4.3, Table 1); a batched
 * plan runs all sets through one chain of launches instead.  The common
 * descriptor supplies precision, basis, kernel, norm, layout, dtypes and
 * flags (its m, n1, n2, strides are ignored).  Each set's outputs have the
 * common layout with row stride n.  All sets use one output tile shape: the
 * descriptor's tile, else the tuned shape of the set with the largest
 * m n^2.  Errors as corr2d_plan, per item; EUNSUPPORTED for interpolation. */
corr2d_status corr2d_batched_plan(corr2d_plan_t* out, const corr2d_desc* common,
                                  const corr2d_item* items, int64_t count);

/* Release a plan (and any graph it instantiated).  NULL is accepted.        */
corr2d_status corr2d_plan_destroy(corr2d_plan_t plan);

/* Device workspace a call needs, in bytes (the caller allocates it; 256-byte
 * alignment required).  It holds the intermediate results of the steps of
 * Sec. 4.2: the reference spectrum (Eq. (ref)), the transform tables and
 * the Fourier-transformed dynamic spectra (Eqs. (disFT), (symmeFT)) as the
 * packed contraction operands, with their scale vectors.  EINVAL for a NULL
 * argument.                                                                  */
corr2d_status corr2d_workspace_bytes(corr2d_plan_t plan, size_t* bytes);

corr2d_status corr2d_plan_get_info(corr2d_plan_t plan, corr2d_plan_info* info);

/* Homocorrelation, the paper's corr2d(Mat1) (Sec. 3, Sec. 4.2), with the
 * interpolation of Sec. 4.1 and the result scaling of Sec. 2 Eqs.
 * (scalesyn), (scaleasyn) when the plan asks for them.
 *   y    device, m x ld_in1 of in_dtype
 *   ref  device, n1 doubles, or NULL for the perturbation mean spectrum
 *   phi, psi  device outputs of out_dtype in out_layout (n1 x n1)
 *   ws   device workspace of ws_bytes >= corr2d_workspace_bytes
 * EINVAL for a NULL y/phi/psi or a plan made for heterocorrelation.          */
corr2d_status corr2d_homo(corr2d_plan_t plan, const void* y, const double* ref,
                          void* phi, void* psi, void* ws, size_t ws_bytes, void* stream);

/* corr2d_homo for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation with no workspace argument.  The library's fixed device
 * scratch of CORR2D_NOALLOC_SCRATCH_BYTES (one copy per GPU, held until the
 * process ends) serves as the workspace; the call makes no hipMalloc,
 * hipFree, hipHostMalloc or other allocating call.
 *   EWORKSPACE   the plan's workspace (corr2d_workspace_bytes) exceeds the
 *                scratch (m = 256, n = 16384 fits in split-BF16, FP32, BF16)
 *   EUNSUPPORTED an interpolation plan (its weights go through pinned memory)
 *   EINVAL       as corr2d_homo
 * Every call on one GPU uses that GPU's scratch: calls that overlap on one
 * GPU (other streams, other threads) race and must be serialized by the
 * caller.  Nothing in the scratch needs clearing between calls: each call
 * writes every scratch byte it reads.                                        */
#define CORR2D_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
corr2d_status corr2d_homo_noalloc(corr2d_plan_t plan, const void* y, const double* ref,
                                  void* phi, void* psi, void* stream);

/* Heterocorrelation, corr2d(Mat1, Mat2) (Sec. 3): two data sets sharing the
 * m perturbation steps.  Psi(nu1, nu2) = Y1^T H Y2 -- the Hilbert transform
 * acts on the second set (Eq. (disHTasyn)).  ref1/ref2 independently NULL for
 * each set's mean.  Outputs are FULL n1 x n2.                                */
corr2d_status corr2d_hetero(corr2d_plan_t plan, const void* y1, const double* ref1,
                            const void* y2, const double* ref2, void* phi, void* psi,
                            void* ws, size_t ws_bytes, void* stream);

/* Batched homocorrelation: corr2d(Mat1) (Sec. 3) of every data set of the
 * plan.  y_base, phi_base, psi_base: device; each set at its item offsets.
 * With neither SEQUENTIAL nor NO_GRAPH the whole batch (prep and one
 * persistent contraction launch) is replayed from a hipGraph
 * the plan captures on first use for these pointers and stream; the job
 * arrays are uploaded from a pinned host buffer that the plan allocates on
 * its first call.  A call with other pointers or another stream than the
 * previous one waits (on the host) for that previous call's job upload
 * before it rewrites the buffer.                                           */
corr2d_status corr2d_batched(corr2d_plan_t plan, const void* y_base, void* phi_base,
                             void* psi_base, void* ws, size_t ws_bytes, void* stream);

/* Measurement hook of the calling thread: when set (hipEvent_t handles
 * passed as void*, either may be NULL), the calling thread's later
 * corr2d_homo and corr2d_hetero calls record `before` on the call's stream
 * immediately before the contraction kernel and `after` immediately after
 * it, so that kernel can be timed alone.  The library keeps the handles
 * (it does not own them) in thread-local storage; pass NULLs to stop.       */
corr2d_status corr2d_set_timing_events(void* before, void* after);

const char* corr2d_status_str(corr2d_status s);

/* Text of the last error on the calling thread ("" if none).                 */
const char* corr2d_last_error(void);

/* Library version string.                                                    */
const char* corr2d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CORR2D_H */
