// api.cpp -- the C ABI of include/corr2d.h: validation, plans (host memory
// only), workspace layout and launch sequences.  Device work is enqueued by
// the launchers of kernels.hip; nothing here computes a correlation value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "corr2d.h"
#include "corr2d_internal.h"
#include "interp.h"
#include "launch.h"
#include "tune.h"

using namespace corr2d;

namespace {

thread_local std::string g_last_error;
// Measurement hook of the calling thread (corr2d_set_timing_events).
thread_local hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr;

corr2d_status fail(corr2d_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
corr2d_status fail(corr2d_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

corr2d_status ok() {
    g_last_error.clear();
    return CORR2D_OK;
}

corr2d_status device_fail(hipError_t e, const char* where) {
    return fail(CORR2D_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Job arrays of a batched call (pinned on the host, copied to the workspace).
struct BlobLayout {
    size_t tables, tstart, qstart, prep, cstart, xstart, corr, tilestart, total;
};

BlobLayout blob_layout(size_t nd, size_t count) {
    BlobLayout b;
    size_t o = 0;
    b.tables = o; o = align256(o + nd * sizeof(TableJob));
    b.tstart = o; o = align256(o + (nd + 1) * sizeof(int32_t));
    b.qstart = o; o = align256(o + (nd + 1) * sizeof(int32_t));
    b.prep = o; o = align256(o + count * sizeof(PrepJob));
    b.cstart = o; o = align256(o + (count + 1) * sizeof(int32_t));
    b.xstart = o; o = align256(o + (count + 1) * sizeof(int32_t));
    b.corr = o; o = align256(o + count * sizeof(CorrJob));
    b.tilestart = o; o = align256(o + (count + 1) * sizeof(int64_t));
    b.total = o;
    return b;
}


constexpr int64_t kMaxM = 4096;          // twiddle table limit of the table kernel
constexpr int64_t kMaxN = (int64_t)1 << 24;

// Geometry of one data set under a precision.
struct Geo {
    int64_t m = 0, n = 0, n_pad = 0;
    int32_t kp = 0, kt = 0, rows_pad = 0;
};

Geo geometry(int64_t m, int64_t n, int prec) {
    Geo g;
    g.m = m;
    g.n = n;
    // the 16-bit formats pair two 128-row panels in one 256-row tile
    g.n_pad = round_up(n, blocked_layout(prec) ? 2 * kNPad : kNPad);
    g.kp = (int32_t)round_up(m, k_align(prec));
    g.kt = (int32_t)round_up(m, kTransformK);
    g.rows_pad = (int32_t)round_up(2 * (int64_t)g.kp, kTransformTile);
    return g;
}

// Workspace regions of one data set (byte offsets from the workspace base).
struct SetLayout {
    size_t ref = 0, yt = 0, sA = 0, sB = 0, A0 = 0, A1 = 0, B0 = 0, B1 = 0;
    bool has_b = false;
};

struct Tile {
    int id = 2, fm = 4, fn = 4;
};

// Tile id 1: 64 x 64 outputs; id 2: 128 x 128, 128 x 64 for FP64 (its
// accumulators are twice as wide), or 256 x 128 for the 16-bit formats
// (LDS-staged kernel, one workgroup per CU); id 3: 128 x 128 of the
// LDS-staged kernel (two workgroups per CU).
Tile tile_from_id(int id, int prec) {
    Tile t;
    t.id = id;
    t.fm = t.fn = (id == 1) ? 2 : 4;
    if (id == 2 && blocked_layout(prec)) t.fm = 8;
    if (id == 2 && prec == CORR2D_PREC_F64) t.fn = 2;   // FP64: 128 x 64
    return t;
}

}  // namespace

struct corr2d_plan_s {
    corr2d_desc d;
    bool batched = false;
    bool hetero = false;
    bool scale = false;
    float qhalf = 1.0f;
    double c = 0.0;           // per data set for single plans
    double boundA = 1.0, boundB = 1.2;
    Tile tile;
    int group = 8;
    // single / hetero
    Geo g1, g2;
    bool fft = false;         // radix FFT transform (else the table product)
    // table product with the centring fused into it (not FP64, kt small enough
    // for the centred columns to stay in LDS): no separate centring launch
    bool fused_center = false;
    // row-selective split: energy partials per operand, the selection record
    bool rowsel = false;
    double fmax = 0.0;
    size_t energy_off[3] = {0, 0, 0};
    size_t sel_off = 0;
    size_t table_off = 0;
    SetLayout s1, s2;
    size_t ws_bytes = 0;
    int64_t ntiles = 0;
    // batched
    struct Item {
        corr2d_item it;
        Geo g;
        SetLayout s;
        size_t table_off;
        double c;
        Tile tile;
        int64_t ntiles;
    };
    std::vector<Item> items;
    std::vector<int> order;             // items by tile shape, then in descending cost
    // one persistent launch per tile shape: items order[first, first + count)
    struct Group {
        Tile tile;
        int first = 0, count = 0;
        int64_t tiles = 0;
    };
    std::vector<Group> groups;
    std::vector<int64_t> distinct_m;
    std::vector<size_t> table_of_m;
    size_t jobs_off = 0, jobs_bytes = 0;
    size_t counter_off = 0;
    int64_t total_tiles = 0;
    int64_t out_elements = 0;
    // interpolation onto the equidistant perturbation grid
    bool interp = false;
    InterpWeights iw;
    size_t iw_off = 0, iw_bytes = 0, yi1_off = 0, yi2_off = 0;
    void* iw_blob = nullptr;   // pinned copy of W and the block ranges (first call)
    std::mutex mu;
    // graph cache (one entry)
    struct GraphKey {
        const void* y = nullptr;
        void* phi = nullptr;
        void* psi = nullptr;
        void* ws = nullptr;
        void* stream = nullptr;
        bool operator==(const GraphKey& o) const {
            return y == o.y && phi == o.phi && psi == o.psi && ws == o.ws && stream == o.stream;
        }
    } key;
    bool have_graph = false;
    hipGraphExec_t gexec = nullptr;
    void* host_blob = nullptr;          // pinned host copy of the job arrays
    // recorded on the call's stream after the last enqueued reader of
    // host_blob (the job upload, inside the graph or not)
    hipEvent_t blob_done = nullptr;
    bool blob_recorded = false;
    bool blob_valid = false;
    GraphKey blob_key;
};

namespace {

bool valid_enum(int v, int lo, int hi) { return v >= lo && v <= hi; }

corr2d_status check_common(const corr2d_desc* d) {
    if (!valid_enum(d->in_dtype, 0, 1) || !valid_enum(d->out_dtype, 0, 1))
        return fail(CORR2D_EINVAL, "in_dtype/out_dtype must be CORR2D_DTYPE_F64 or _F32");
    if (!valid_enum(d->prec, 0, 6)) return fail(CORR2D_EINVAL, "unknown prec %d", d->prec);
    if (!valid_enum(d->basis, 0, 2)) return fail(CORR2D_EINVAL, "unknown basis %d", d->basis);
    if (!valid_enum(d->hilbert, 0, 2)) return fail(CORR2D_EINVAL, "unknown hilbert %d", d->hilbert);
    if (d->hilbert == CORR2D_HILBERT_R_COMPAT && d->basis == CORR2D_BASIS_TIME)
        return fail(CORR2D_EUNSUPPORTED, "the R-compatible bin list needs the Fourier basis");
    if (!valid_enum(d->norm_mode, 0, 2)) return fail(CORR2D_EINVAL, "unknown norm_mode %d", d->norm_mode);
    if (!valid_enum(d->out_layout, 0, 2)) return fail(CORR2D_EINVAL, "unknown out_layout %d", d->out_layout);
    if (d->norm_mode == CORR2D_NORM_CUSTOM && !std::isfinite(d->norm_value))
        return fail(CORR2D_EINVAL, "CUSTOM norm needs a finite norm_value");
    if (!std::isfinite(d->scale_alpha))
        return fail(CORR2D_EINVAL, "scale_alpha must be finite");
    if (!valid_enum(d->interp, 0, 2)) return fail(CORR2D_EINVAL, "unknown interp %d", d->interp);
    if (d->interp != CORR2D_INTERP_NONE) {
        if (!d->t_in) return fail(CORR2D_EINVAL, "interpolation needs t_in");
        if (d->m_in < 2 || d->m_in > kMaxM)
            return fail(CORR2D_EINVAL, "m_in = %lld out of range", (long long)d->m_in);
        for (int64_t i = 0; i < d->m_in; ++i) {
            if (!std::isfinite(d->t_in[i])) return fail(CORR2D_EINVAL, "t_in[%lld] is not finite", (long long)i);
            if (i > 0 && !(d->t_in[i] > d->t_in[i - 1]))
                return fail(CORR2D_EINVAL, "t_in must be strictly increasing (t_in[%lld])", (long long)i);
        }
    }
    if (d->flags & ~0x3fu) return fail(CORR2D_EINVAL, "unknown flag bits 0x%x", d->flags);
    if (!std::isfinite(d->split_tol) || d->split_tol < 0.0)
        return fail(CORR2D_EINVAL, "split_tol must be finite and >= 0");
    if ((d->flags & CORR2D_FLAG_SPLIT_ROWS) && d->prec != CORR2D_PREC_SPLIT_BF16 &&
        d->prec != CORR2D_PREC_SPLIT_F16)
        return fail(CORR2D_EUNSUPPORTED, "the row-selective split needs a split format");
    if ((d->flags & CORR2D_FLAG_SPLIT_ROWS) && d->basis == CORR2D_BASIS_TIME)
        return fail(CORR2D_EUNSUPPORTED, "the row-selective split works on the Fourier rows");
    if (d->prec == CORR2D_PREC_FP8_E4M3 && (d->flags & CORR2D_FLAG_NO_PER_BAND_SCALE))
        return fail(CORR2D_EUNSUPPORTED, "FP8 e4m3 requires per-band scaling (range 448)");
    if (d->prec == CORR2D_PREC_SPLIT_F16 && (d->flags & CORR2D_FLAG_NO_PER_BAND_SCALE))
        return fail(CORR2D_EUNSUPPORTED, "split FP16 requires per-band scaling (range 65504)");
    if (d->tile < 0 || d->tile > 3)
        return fail(CORR2D_EINVAL, "unknown tile id %d", d->tile);
    if (d->tile == 3 && !blocked_layout(d->prec))
        return fail(CORR2D_EUNSUPPORTED, "tile 3 (128x128, LDS-staged) is built for the 16-bit formats only");
    if (d->tile == 1 && blocked_layout(d->prec))
        return fail(CORR2D_EUNSUPPORTED, "tile 1 (64x64) is not built for the 16-bit formats");
    return CORR2D_OK;
}

// CORR2D_BASIS_AUTO: the time basis, where the operands' rounding errors
// spread over all m products of a sum instead of concentrating in the few
// Fourier rows that carry a band spectrum's energy.  Measured on the band
// workloads (relative Frobenius error over the full matrices, Fourier ->
// time): split-BF16 4.7e-6 -> 6.7e-7 at m = 256 and 5.4e-5 -> 9.1e-6 on the
// worst of the 256 batched data sets, FP16 3.1e-4 -> 4.4e-5, FP8 4.0e-2 ->
// 7.1e-3, plain BF16 2.5e-3 -> 3.5e-4, FP32 4.4e-7 -> 2.7e-7, FP64 equal;
// the contraction costs the same.  The Fourier basis where the method
// needs it: the R bin list, and the row-selective split (it picks Fourier
// rows).
int resolve_basis(const corr2d_desc* d) {
    if (d->basis != CORR2D_BASIS_AUTO) return d->basis;
    if (d->hilbert == CORR2D_HILBERT_R_COMPAT || (d->flags & CORR2D_FLAG_SPLIT_ROWS)) return CORR2D_BASIS_FOURIER;
    return CORR2D_BASIS_TIME;
}

double norm_cF(const corr2d_desc* d, int64_t m) {
    switch (d->norm_mode) {
    case CORR2D_NORM_PAPER: return 1.0 / (M_PI * (double)(m - 1));
    case CORR2D_NORM_CUSTOM: return d->norm_value;
    default: return 1.0 / ((double)m * (double)(m - 1));
    }
}

// The contraction's operands are Fourier coefficients (A = Q Yc, Q^T Q = m I)
// or the dynamic spectra themselves; cF multiplies the Fourier sum, which is
// m times the time-basis sum.
double contraction_factor(const corr2d_desc* d, int64_t m) {
    const double cF = norm_cF(d, m);
    return d->basis == CORR2D_BASIS_TIME ? cF * (double)m : cF;
}

void set_scaling(corr2d_plan_s* p) {
    const int prec = p->d.prec;
    p->scale = false;
    if (prec == CORR2D_PREC_FP8_E4M3) {
        p->scale = true;
        p->qhalf = 224.0f;
    } else if (prec == CORR2D_PREC_F16) {
        p->scale = !(p->d.flags & CORR2D_FLAG_NO_PER_BAND_SCALE);
        p->qhalf = 32752.0f;
    } else if (prec == CORR2D_PREC_SPLIT_F16) {
        p->scale = true;
        p->qhalf = 32752.0f;
    }
}

double bound_a(const corr2d_desc* d, int64_t m) {
    return d->basis == CORR2D_BASIS_TIME ? 1.0 : std::sqrt((double)m);
}

// Layout of one data set's workspace regions, appended at *off.
// The centred spectra (yt) are needed by the table-product transform only;
// the radix FFT transform centres in registers and LDS (need_yt false).
SetLayout layout_set(const Geo& g, int prec, bool t64, bool need_b, bool need_yt, size_t* off) {
    SetLayout s;
    const size_t tsz = t64 ? 8 : 4;
    const size_t esz = (size_t)elem_bytes(prec);
    const size_t plane = (size_t)g.n_pad * g.kp * esz;
    s.ref = *off; *off = align256(*off + (size_t)g.n_pad * sizeof(double));
    s.yt = *off;
    if (need_yt) *off = align256(*off + (size_t)g.n_pad * g.kt * tsz);
    s.sA = *off; *off = align256(*off + (size_t)g.n_pad * 4);
    s.A0 = *off; *off = align256(*off + plane);
    if (planes(prec) == 2) { s.A1 = *off; *off = align256(*off + plane); }
    s.has_b = need_b;
    if (need_b) {
        s.sB = *off; *off = align256(*off + (size_t)g.n_pad * 4);
        s.B0 = *off; *off = align256(*off + plane);
        if (planes(prec) == 2) { s.B1 = *off; *off = align256(*off + plane); }
    }
    return s;
}

size_t table_bytes(const Geo& g, bool t64) { return (size_t)g.rows_pad * g.kt * (t64 ? 8 : 4); }

template <class T>
T* at(void* ws, size_t off) {
    return (T*)((char*)ws + off);
}

TableJob make_table_job(const corr2d_plan_s* p, const Geo& g, void* ws, size_t off) {
    TableJob t{};
    t.m = g.m;
    t.kp = g.kp;
    t.kt = g.kt;
    t.rows_pad = g.rows_pad;
    t.basis = p->d.basis;
    t.hilbert = p->d.hilbert;
    t.f64 = p->d.prec == CORR2D_PREC_F64;
    t.table = at<char>(ws, off);
    return t;
}

int table_blocks(const Geo& g) { return (int)(((int64_t)g.rows_pad * g.kt + 255) / 256); }

PrepJob make_prep_job(const corr2d_plan_s* p, const Geo& g, const SetLayout& s, const void* y,
                      int64_t ld, const double* ref, void* ws, size_t table_off) {
    PrepJob j{};
    j.y = y;
    j.ref = ref;
    j.ld = ld;
    j.m = g.m;
    j.n = g.n;
    j.n_pad = g.n_pad;
    j.kp = g.kp;
    j.kt = g.kt;
    j.rows_pad = g.rows_pad;
    j.in_f64 = p->d.in_dtype == CORR2D_DTYPE_F64;
    j.t_f64 = p->d.prec == CORR2D_PREC_F64;
    j.prec = p->d.prec;
    j.need_b = s.has_b;
    j.scale = p->scale;
    j.qhalf = p->qhalf;
    j.boundA = bound_a(&p->d, g.m);
    j.boundB = 1.2 * j.boundA;
    j.yt = at<char>(ws, s.yt);
    j.table = at<char>(ws, table_off);
    j.sA = at<float>(ws, s.sA);
    j.sB = s.has_b ? at<float>(ws, s.sB) : nullptr;
    j.A0 = at<char>(ws, s.A0);
    j.A1 = s.A1 ? at<char>(ws, s.A1) : nullptr;
    j.B0 = s.has_b ? at<char>(ws, s.B0) : nullptr;
    j.B1 = (s.has_b && s.B1) ? at<char>(ws, s.B1) : nullptr;
    j.alpha = p->d.scale_alpha;
    j.hilbert = p->d.hilbert;
    j.basis = p->d.basis;
    j.ref_out = at<double>(ws, s.ref);
    return j;
}

int center_blocks(const Geo& g) { return (int)(g.n_pad / kCenterCols); }
// Workgroups of the transform GEMM: FP64 uses 64 x 64 tiles, the FP32
// kernel 64 x 256 (spectral points x transform rows).
int transform_blocks(const Geo& g, int prec) {
    if (prec == CORR2D_PREC_F64) return (int)((g.n_pad / kTransformTile) * (g.rows_pad / kTransformTile));
    return (int)((g.n_pad / 64) * ((g.rows_pad + 255) / 256));
}
// Workgroups of the transform launch: the fused centring kernel has one per
// 64 spectral points (it runs the row tiles in turn).
int prep_blocks(const Geo& g, int prec, bool fused) {
    return fused ? (int)(g.n_pad / 64) : transform_blocks(g, prec);
}

// The radix FFT transform (FP64 for the FP64 path, else FP32) serves
// power-of-two m in [128, 1024]: the Fourier basis, and the time basis with
// Noda's kernel (B = N Yc as an FFT correlation).  A flag asks for the
// table product everywhere.
bool use_fft(const corr2d_desc* d, int64_t m) {
    if (d->flags & CORR2D_FLAG_TRANSFORM_MATMUL) return false;
    if (d->basis == CORR2D_BASIS_TIME && d->hilbert != CORR2D_HILBERT_NODA) return false;
    return m >= 128 && m <= 1024 && (m & (m - 1)) == 0;
}
int fft_log2(int64_t m) {
    int l = 0;
    while (((int64_t)1 << l) < 2 * m) ++l;
    return l;
}
int fft_blocks(const Geo& g) { return (int)(g.n_pad / fft_points((int)(2 * g.m))); }

// The Q N rows of the table (Fourier basis, Noda's kernel) come from their
// own kernel.
bool needs_qn(const corr2d_plan_s* p) {
    return p->d.basis == CORR2D_BASIS_FOURIER && p->d.hilbert == CORR2D_HILBERT_NODA;
}

// CORR2D_LOG set (and not "0") in the environment: one line per plan on
// stderr with the decisions the library took.
bool log_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("CORR2D_LOG");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}

const char* prec_name(int prec) {
    static const char* names[] = {"f64", "f32", "split_bf16", "bf16", "f16", "fp8_e4m3", "split_f16"};
    return prec >= 0 && prec < 7 ? names[prec] : "?";
}

// Table-product plans with m <= kPrepMergeMaxM build the table and centre
// the spectra in one launch (after the optional resampling); the others
// launch their tables first (FFT plans centre inside the transform).
bool merged_prep(const corr2d_plan_s* p) { return !p->fft && p->g1.m <= kPrepMergeMaxM; }

// Tables of a single or heterocorrelation plan: the DFT table (and its Q N
// rows), or the twiddles and Noda multiplier of the radix FFT transform.
hipError_t launch_prep_tables(const corr2d_plan_s* p, const TableSrcInline& ts, hipStream_t s) {
    if (p->fft) return launch_fft_tables(ts, p->g1.m, s);
    hipError_t e = launch_tables(ts, ts.blocks0, p->g1.m, s);
    if (e == hipSuccess && needs_qn(p)) e = launch_tables_qn(ts, qn_blocks(p->g1.m), p->g1.m, s);
    return e;
}

// Tiles of the upper triangle when a row tile is R column tiles tall: row
// tile I pairs with column tiles J >= R I of the R T column tiles.
int64_t triangle_tiles(int64_t T, int64_t R) { return R * T * (T + 1) / 2; }

// Fraction of the hi*hi rounding-error energy the rows without the low
// plane may hold: with RNE halves of unit roundoff u (2^-8 BF16, 2^-11
// FP16) the rounding errors are about uniform, rms u/sqrt(3); the error
// energy of the products left to hi*hi, 2 (u/sqrt(3))^2 times their share
// f of sum_k E_k^2, over ||Phi||_F^2 >= sum_k E_k^2 (the diagonal of the
// rows' Gram matrix) gives a relative error of (u/sqrt(3)) sqrt(2 f).  The
// rounding errors of band spectra's Fourier rows are not independent of the
// values (on the m = 256, n = 16384 band workload the rows left to hi*hi in
// split BF16 added twice the modelled error), so the model is held to an
// eighth of the target eps (the kept products, the transform and the FP32
// accumulation take the rest):  f = (eps / (8 u / sqrt(3)))^2 / 2.
double split_fmax(const corr2d_desc* d) {
    const double eps = d->split_tol > 0.0 ? d->split_tol : 1e-5;
    const double u = d->prec == CORR2D_PREC_SPLIT_F16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
    const double r = eps / (8.0 * u / std::sqrt(3.0));
    return 0.5 * r * r;
}

// Energy and selection launches of a row-selective call: operand 0 the
// left A (set 1), 1 the right A (set 2; none for a homocorrelation), 2 the
// right B.
hipError_t launch_selection(const corr2d_plan_s* p, void* ws, hipStream_t s) {
    SelJob J{};
    const SetLayout& r = p->hetero ? p->s2 : p->s1;
    const Geo& gr = p->hetero ? p->g2 : p->g1;
    J.X[0] = at<char>(ws, p->s1.A0);
    J.X[1] = p->hetero ? at<char>(ws, p->s2.A0) : J.X[0];
    J.X[2] = at<char>(ws, r.B0);
    J.s[0] = p->scale ? at<float>(ws, p->s1.sA) : nullptr;
    J.s[1] = p->scale ? at<float>(ws, p->hetero ? p->s2.sA : p->s1.sA) : nullptr;
    J.s[2] = p->scale ? at<float>(ws, r.sB) : nullptr;
    for (int o = 0; o < 3; ++o) J.part[o] = at<float>(ws, p->energy_off[o]);
    J.panels[0] = (int32_t)(p->g1.n_pad / 128);
    J.panels[1] = p->hetero ? (int32_t)(p->g2.n_pad / 128) : 0;
    J.panels[2] = (int32_t)(gr.n_pad / 128);
    J.kp = p->g1.kp;
    J.prec = p->d.prec;
    J.fmax = p->fmax;
    J.sel = at<int32_t>(ws, p->sel_off);
    return launch_row_select(J, s);
}

CorrJob make_corr_job(const corr2d_plan_s* p, const Geo& g1, const SetLayout& s1, const Geo& g2,
                      const SetLayout& s2, void* ws, void* phi, void* psi, bool homo, double c,
                      const Tile& tile, int64_t ld_out, int layout) {
    CorrJob C{};
    C.L0 = at<char>(ws, s1.A0);
    C.L1 = s1.A1 ? at<char>(ws, s1.A1) : nullptr;
    C.RA0 = at<char>(ws, s2.A0);
    C.RA1 = s2.A1 ? at<char>(ws, s2.A1) : nullptr;
    C.RB0 = at<char>(ws, s2.B0);
    C.RB1 = s2.B1 ? at<char>(ws, s2.B1) : nullptr;
    C.sL = at<float>(ws, s1.sA);
    C.sRA = at<float>(ws, s2.sA);
    C.sRB = at<float>(ws, s2.sB);
    C.phi = phi;
    C.psi = psi;
    C.n1 = g1.n;
    C.n2 = g2.n;
    C.ld_out = ld_out;
    C.kp = g1.kp;
    C.tiles_i = (int32_t)(g1.n_pad / (32 * tile.fm));
    C.tiles_j = (int32_t)(g2.n_pad / (32 * tile.fn));
    C.ratio = tile.fm / tile.fn;
    C.homo = homo;
    C.layout = layout;
    C.out_f64 = p->d.out_dtype == CORR2D_DTYPE_F64;
    C.group = p->group;
    C.scaled = p->scale;
    C.ntiles = homo ? triangle_tiles(C.tiles_i, C.ratio) : (int64_t)C.tiles_i * C.tiles_j;
    C.c = c;
    // both output planes of this call (batched plans write far more); in
    // floating point, as a caller's row stride can be arbitrarily large
    const double rows = (double)g1.n;
    const double elems = (!homo || layout == L_FULL) ? rows * (double)ld_out : rows * (rows + 32.0) / 2.0;
    const double out_bytes = 2.0 * elems * (C.out_f64 ? 8.0 : 4.0);
    C.store_near = !p->batched && out_bytes <= (double)kNearStoreBytes;
    return C;
}

Tile choose_tile(const corr2d_desc* d, int64_t m, int64_t n) {
    if (d->tile) return tile_from_id(d->tile, d->prec);
    return tile_from_id(tune_lookup(d->prec, m, n), d->prec);
}

corr2d_status check_ws(const corr2d_plan_s* p, void* ws, size_t ws_bytes) {
    if (!ws) return fail(CORR2D_EWORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) & 255) return fail(CORR2D_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < p->ws_bytes)
        return fail(CORR2D_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                    ws_bytes, p->ws_bytes);
    return CORR2D_OK;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void corr2d_desc_init(corr2d_desc* d) {
    if (!d) return;
    std::memset(d, 0, sizeof *d);
    d->in_dtype = CORR2D_DTYPE_F64;
    d->out_dtype = CORR2D_DTYPE_F32;
    d->prec = CORR2D_PREC_SPLIT_BF16;
    d->basis = CORR2D_BASIS_AUTO;
    d->hilbert = CORR2D_HILBERT_NODA;
    d->norm_mode = CORR2D_NORM_NODA;
    d->out_layout = CORR2D_LAYOUT_FULL;
}

const char* corr2d_status_str(corr2d_status s) {
    switch (s) {
    case CORR2D_OK: return "CORR2D_OK";
    case CORR2D_EINVAL: return "CORR2D_EINVAL";
    case CORR2D_EWORKSPACE: return "CORR2D_EWORKSPACE";
    case CORR2D_EUNSUPPORTED: return "CORR2D_EUNSUPPORTED";
    case CORR2D_EDEVICE: return "CORR2D_EDEVICE";
    case CORR2D_ENOMEM: return "CORR2D_ENOMEM";
    }
    return "CORR2D_UNKNOWN";
}

const char* corr2d_last_error(void) { return g_last_error.c_str(); }

const char* corr2d_version(void) { return "corr2d-mi355x 0.1 (gfx950)"; }

corr2d_status corr2d_plan(corr2d_plan_t* out, const corr2d_desc* d) {
    if (!out || !d) return fail(CORR2D_EINVAL, "NULL plan or descriptor");
    *out = nullptr;
    corr2d_status st = check_common(d);
    if (st != CORR2D_OK) return st;
    if (d->m < 2) return fail(CORR2D_EINVAL, "m = %lld: at least 2 perturbation steps are needed", (long long)d->m);
    if (d->m > kMaxM) return fail(CORR2D_EUNSUPPORTED, "m = %lld exceeds %lld", (long long)d->m, (long long)kMaxM);
    if (d->n1 < 1 || d->n1 > kMaxN) return fail(CORR2D_EINVAL, "n1 = %lld out of range", (long long)d->n1);
    if (d->n2 < 0 || d->n2 > kMaxN) return fail(CORR2D_EINVAL, "n2 = %lld out of range", (long long)d->n2);
    const bool hetero = d->n2 > 0;
    if (hetero && d->out_layout != CORR2D_LAYOUT_FULL)
        return fail(CORR2D_EINVAL, "upper-triangle outputs are defined for homocorrelation only");
    const int64_t ld1 = d->ld_in1 ? d->ld_in1 : d->n1;
    const int64_t ld2 = d->ld_in2 ? d->ld_in2 : d->n2;
    if (ld1 < d->n1) return fail(CORR2D_EINVAL, "ld_in1 < n1");
    if (hetero && ld2 < d->n2) return fail(CORR2D_EINVAL, "ld_in2 < n2");
    const int64_t cols = hetero ? d->n2 : d->n1;
    const int64_t ldo = d->ld_out ? d->ld_out : cols;
    if (ldo < cols) return fail(CORR2D_EINVAL, "ld_out smaller than the number of output columns");

    corr2d_plan_s* p = new (std::nothrow) corr2d_plan_s;
    if (!p) return fail(CORR2D_ENOMEM, "host allocation of the plan failed");
    p->d = *d;
    p->d.basis = resolve_basis(d);
    p->d.ld_in1 = ld1;
    p->d.ld_in2 = hetero ? ld2 : 0;
    p->d.ld_out = ldo;
    p->hetero = hetero;
    set_scaling(p);
    p->c = contraction_factor(&p->d, d->m);
    p->tile = choose_tile(d, d->m, hetero ? std::max(d->n1, d->n2) : d->n1);
    if (!corr_variant_supported(d->prec, p->tile.fm, p->tile.fn)) {
        delete p;
        return fail(CORR2D_EUNSUPPORTED, "tile %d is not built for precision %d", p->tile.id, d->prec);
    }
    const bool t64 = d->prec == CORR2D_PREC_F64;
    p->g1 = geometry(d->m, d->n1, d->prec);
    p->fft = use_fft(&p->d, d->m);
    // a single call fuses the centring only when the transform has enough
    // work to fill the GPU: at least 512 tiles of 64 spectral points x 256
    // transform rows (the separate centring has a workgroup per 32 points);
    // at m = 64, n = 4096 (64 tiles) fusing cost 3 us per call
    const int fused_blocks = transform_blocks(p->g1, d->prec) +
                             (hetero ? transform_blocks(geometry(d->m, d->n2, d->prec), d->prec) : 0);
    p->fused_center = !p->fft && d->prec != CORR2D_PREC_F64 && p->g1.kt <= kFusedTransformMaxK &&
                      fused_blocks >= kFusedMinBlocks;
    size_t off = 0;
    p->table_off = off;
    off = align256(off + table_bytes(p->g1, t64));
    if (!hetero) {
        p->s1 = layout_set(p->g1, d->prec, t64, true, !p->fft, &off);
        const int64_t T = p->g1.n_pad / (32 * p->tile.fm);
        p->ntiles = triangle_tiles(T, p->tile.fm / p->tile.fn);
    } else {
        p->g2 = geometry(d->m, d->n2, d->prec);
        p->s1 = layout_set(p->g1, d->prec, t64, false, !p->fft, &off);
        p->s2 = layout_set(p->g2, d->prec, t64, true, !p->fft, &off);
        p->ntiles = (p->g1.n_pad / (32 * p->tile.fm)) * (p->g2.n_pad / (32 * p->tile.fn));
    }
    if (d->flags & CORR2D_FLAG_SPLIT_ROWS) {
        if (p->d.basis != CORR2D_BASIS_FOURIER) {
            delete p;
            return fail(CORR2D_EUNSUPPORTED, "the row-selective split works on the Fourier rows");
        }
        if (p->g1.kp > 16 * kMaxSelBlocks) {
            delete p;
            return fail(CORR2D_EUNSUPPORTED, "the row-selective split orders at most %d K blocks (m <= %d)",
                        kMaxSelBlocks, 16 * kMaxSelBlocks);
        }
        p->rowsel = true;
        p->fmax = split_fmax(&p->d);
        const int64_t np0 = sel_groups((int)(p->g1.n_pad / 128));
        const int64_t np2 = sel_groups((int)((hetero ? p->g2.n_pad : p->g1.n_pad) / 128));
        const int64_t np[3] = {np0, hetero ? np2 : 0, np2};
        for (int o = 0; o < 3; ++o) {
            p->energy_off[o] = off;
            off = align256(off + (size_t)std::max<int64_t>(np[o], 1) * p->g1.kp * sizeof(float));
        }
        p->sel_off = off;
        off = align256(off + (1 + kMaxSelBlocks) * sizeof(int32_t));
    }
    if (d->interp != CORR2D_INTERP_NONE) {
        // weights of the resampling (FP64, host), uploaded with every call;
        // the resampled spectra live in the workspace
        p->interp = true;
        p->d.t_in = nullptr;   // the plan keeps no caller pointer
        if (!build_interp_weights(d->t_in, d->m_in, d->m, d->interp, p->iw)) {
            delete p;
            return fail(CORR2D_EINVAL, "interpolation weights are not finite");
        }
        p->iw_bytes = align256(p->iw.W.size() * sizeof(double)) + p->iw.block_range.size() * sizeof(int32_t);
        p->iw_off = off;
        off = align256(off + p->iw_bytes);
        p->yi1_off = off;
        off = align256(off + (size_t)d->m * (size_t)p->g1.n_pad * sizeof(double));
        if (hetero) {
            p->yi2_off = off;
            off = align256(off + (size_t)d->m * (size_t)p->g2.n_pad * sizeof(double));
        }
    }
    p->ws_bytes = off;
    if (log_enabled())
        std::fprintf(stderr,
                     "corr2d: plan %s m=%lld n1=%lld n2=%lld layout=%d tile=%d (%dx%d) tiles=%lld "
                     "transform=%s prep_launches=%d per_band_scale=%d row_select=%d workspace=%zu B tune: %s\n",
                     prec_name(d->prec), (long long)d->m, (long long)d->n1, (long long)d->n2, d->out_layout,
                     p->tile.id, 32 * p->tile.fm, 32 * p->tile.fn, (long long)p->ntiles,
                     p->fft ? "radix FFT" : (p->fused_center ? "DFT table product, centring fused" : "DFT table product"),
                     p->fft ? 2 : (merged_prep(p) ? 2 : (needs_qn(p) ? 4 : 3) - (p->fused_center ? 1 : 0)),
                     (int)p->scale, (int)p->rowsel, p->ws_bytes, tune_source());
    *out = p;
    return ok();
}

corr2d_status corr2d_batched_plan(corr2d_plan_t* out, const corr2d_desc* common,
                                  const corr2d_item* items, int64_t count) {
    if (!out || !common || !items) return fail(CORR2D_EINVAL, "NULL argument");
    *out = nullptr;
    if (count < 1 || count > (1 << 20)) return fail(CORR2D_EINVAL, "count = %lld out of range", (long long)count);
    corr2d_status st = check_common(common);
    if (st != CORR2D_OK) return st;
    if (common->interp != CORR2D_INTERP_NONE)
        return fail(CORR2D_EUNSUPPORTED, "interpolation is not available for batched plans");
    if (common->flags & CORR2D_FLAG_SPLIT_ROWS)
        return fail(CORR2D_EUNSUPPORTED, "the row-selective split is not available for batched plans");
    for (int64_t i = 0; i < count; ++i) {
        const corr2d_item& it = items[i];
        if (it.m < 2 || it.m > kMaxM) return fail(CORR2D_EINVAL, "item %lld: m = %lld out of range", (long long)i, (long long)it.m);
        if (it.n < 1 || it.n > kMaxN) return fail(CORR2D_EINVAL, "item %lld: n = %lld out of range", (long long)i, (long long)it.n);
        if (it.ld_in != 0 && it.ld_in < it.n) return fail(CORR2D_EINVAL, "item %lld: ld_in < n", (long long)i);
        if (it.in_offset < 0 || it.out_offset < 0) return fail(CORR2D_EINVAL, "item %lld: negative offset", (long long)i);
    }
    corr2d_plan_s* p = new (std::nothrow) corr2d_plan_s;
    if (!p) return fail(CORR2D_ENOMEM, "host allocation of the plan failed");
    p->d = *common;
    p->d.basis = resolve_basis(common);
    p->batched = true;
    set_scaling(p);
    const bool t64 = common->prec == CORR2D_PREC_F64;
    size_t off = 0;
    // tables per distinct m
    for (int64_t i = 0; i < count; ++i) {
        if (std::find(p->distinct_m.begin(), p->distinct_m.end(), items[i].m) == p->distinct_m.end())
            p->distinct_m.push_back(items[i].m);
    }
    for (int64_t m : p->distinct_m) {
        p->table_of_m.push_back(off);
        off = align256(off + table_bytes(geometry(m, 1, common->prec), t64));
    }
    // One tile shape for the whole batch (unless the descriptor fixes one):
    // the tuned shape of the data set with the most work (m n^2), so that
    // every tile goes through one persistent launch.  Per-set shapes would
    // split the batch into one launch per shape, run back to back, each
    // with its own ramp and tail (the 256-set FP32 batch: 17.8 ms with two
    // launches, 17.45 ms with one).
    corr2d_desc batch_desc = *common;
    if (batch_desc.tile == 0) {
        int64_t big = 0;
        for (int64_t i = 1; i < count; ++i) {
            const double wi = (double)items[i].m * (double)items[i].n * (double)items[i].n;
            const double wb = (double)items[big].m * (double)items[big].n * (double)items[big].n;
            if (wi > wb) big = i;
        }
        batch_desc.tile = choose_tile(common, items[big].m, items[big].n).id;
    }
    p->items.resize(count);
    p->out_elements = 0;
    for (int64_t i = 0; i < count; ++i) {
        auto& I = p->items[i];
        I.it = items[i];
        if (I.it.ld_in == 0) I.it.ld_in = I.it.n;
        I.g = geometry(I.it.m, I.it.n, common->prec);
        I.s = layout_set(I.g, common->prec, t64, true, true, &off);
        const size_t mi = std::find(p->distinct_m.begin(), p->distinct_m.end(), I.it.m) - p->distinct_m.begin();
        I.table_off = p->table_of_m[mi];
        I.c = contraction_factor(&p->d, I.it.m);
        I.tile = choose_tile(&batch_desc, I.it.m, I.it.n);
        if (!corr_variant_supported(common->prec, I.tile.fm, I.tile.fn)) {
            delete p;
            return fail(CORR2D_EUNSUPPORTED, "tile %d is not built for precision %d", I.tile.id, common->prec);
        }
        I.ntiles = triangle_tiles(I.g.n_pad / (32 * I.tile.fm), I.tile.fm / I.tile.fn);
        const int64_t outn = common->out_layout == CORR2D_LAYOUT_UPPER_PACKED
                                 ? I.it.n * (I.it.n + 1) / 2
                             : common->out_layout == CORR2D_LAYOUT_UPPER_ALIGNED
                                 ? corr2d_upper_aligned_elements(I.it.n)
                                 : I.it.n * I.it.n;
        p->out_elements = std::max(p->out_elements, I.it.out_offset + outn);
    }
    p->fused_center = common->prec != CORR2D_PREC_F64;
    for (const auto& I : p->items) p->fused_center = p->fused_center && I.g.kt <= kFusedTransformMaxK;
    // grouped by tile shape, each group in descending cost order (longest
    // processing time first)
    p->order.resize(count);
    for (int64_t i = 0; i < count; ++i) p->order[i] = (int)i;
    std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) {
        const auto& A = p->items[a];
        const auto& B = p->items[b];
        if (A.tile.id != B.tile.id) return A.tile.id < B.tile.id;
        return (double)A.g.kp * A.ntiles * A.tile.fm * A.tile.fn >
               (double)B.g.kp * B.ntiles * B.tile.fm * B.tile.fn;
    });
    p->total_tiles = 0;
    for (auto& I : p->items) p->total_tiles += I.ntiles;
    for (int64_t r = 0; r < count; ++r) {
        const auto& I = p->items[p->order[r]];
        if (p->groups.empty() || p->groups.back().tile.id != I.tile.id) {
            corr2d_plan_s::Group gr;
            gr.tile = I.tile;
            gr.first = (int)r;
            p->groups.push_back(gr);
        }
        p->groups.back().count += 1;
        p->groups.back().tiles += I.ntiles;
    }
    // the plan reports the shape that covers the most output tiles
    p->tile = p->groups[0].tile;
    int64_t best = -1;
    for (const auto& gr : p->groups)
        if (gr.tiles > best) { best = gr.tiles; p->tile = gr.tile; }
    // job arrays: tables, prep, corr, block starts, tile starts
    const size_t nd = p->distinct_m.size();
    p->jobs_bytes = blob_layout(nd, (size_t)count).total;
    p->jobs_off = off;
    off = align256(off + p->jobs_bytes);
    p->counter_off = off;
    off = align256(off + 256);
    p->ws_bytes = off;
    if (log_enabled()) {
        std::fprintf(stderr, "corr2d: batched plan %s items=%lld distinct_m=%zu tiles=%lld out_elements=%lld "
                             "centring=%s workspace=%zu B tune: %s\n",
                     prec_name(common->prec), (long long)count, p->distinct_m.size(), (long long)p->total_tiles,
                     (long long)p->out_elements, p->fused_center ? "fused" : "separate", p->ws_bytes, tune_source());
        for (const auto& gr : p->groups)
            std::fprintf(stderr, "corr2d:   tile %d (%dx%d): %d data sets, %lld tiles, one persistent launch\n",
                         gr.tile.id, 32 * gr.tile.fm, 32 * gr.tile.fn, gr.count, (long long)gr.tiles);
    }
    *out = p;
    return ok();
}

corr2d_status corr2d_plan_destroy(corr2d_plan_t p) {
    if (!p) return ok();
    if (p->have_graph && p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->blob_done) {
        if (p->blob_recorded) (void)hipEventSynchronize(p->blob_done);
        (void)hipEventDestroy(p->blob_done);
    }
    if (p->host_blob) (void)hipHostFree(p->host_blob);
    if (p->iw_blob) (void)hipHostFree(p->iw_blob);
    delete p;
    return ok();
}

corr2d_status corr2d_workspace_bytes(corr2d_plan_t p, size_t* bytes) {
    if (!p || !bytes) return fail(CORR2D_EINVAL, "NULL argument");
    *bytes = p->ws_bytes;
    return ok();
}

corr2d_status corr2d_set_timing_events(void* before, void* after) {
    g_ev_before = (hipEvent_t)before;
    g_ev_after = (hipEvent_t)after;
    return ok();
}

corr2d_status corr2d_plan_get_info(corr2d_plan_t p, corr2d_plan_info* info) {
    if (!p || !info) return fail(CORR2D_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->tile = p->tile.id;
    info->tile_m = 32 * p->tile.fm;
    info->tile_n = 32 * p->tile.fn;
    info->per_band_scale = p->scale;
    info->workspace_bytes = p->ws_bytes;
    if (p->batched) {
        info->items = (int64_t)p->items.size();
        info->tiles = p->total_tiles;
        info->out_elements = p->out_elements;
        info->k_pad = 0;
        info->n_pad = 0;
        info->c = 0.0;
    } else {
        info->k_pad = p->g1.kp;
        info->n_pad = p->g1.n_pad;
        info->tiles = p->ntiles;
        info->c = p->c;
        info->transform = p->fft ? 1 : 0;
        info->basis = p->d.basis;
        info->sel_offset = p->rowsel ? p->sel_off : 0;
        info->ref1_offset = p->s1.ref;
        info->ref2_offset = p->hetero ? p->s2.ref : p->s1.ref;
    }
    return ok();
}

namespace {

// Upload the interpolation weights (from a pinned copy made on the first
// call) into the workspace.
corr2d_status upload_interp(corr2d_plan_s* p, void* ws, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lock(p->mu);
        if (!p->iw_blob) {
            void* b = nullptr;
            hipError_t e = hipHostMalloc(&b, p->iw_bytes, hipHostMallocDefault);
            if (e != hipSuccess) return device_fail(e, "pinned interpolation weights");
            std::memcpy(b, p->iw.W.data(), p->iw.W.size() * sizeof(double));
            std::memcpy((char*)b + align256(p->iw.W.size() * sizeof(double)), p->iw.block_range.data(),
                        p->iw.block_range.size() * sizeof(int32_t));
            p->iw_blob = b;
        }
    }
    hipError_t e = hipMemcpyAsync(at<char>(ws, p->iw_off), p->iw_blob, p->iw_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_fail(e, "interpolation weight upload");
    return CORR2D_OK;
}

// Resample one data set (m_in input rows) onto the equidistant grid in the
// workspace; the centring then reads it as FP64 rows of stride n_pad.
corr2d_status resample(const corr2d_plan_s* p, void* ws, const void* y, int64_t ld, const Geo& g,
                       size_t out_off, hipStream_t s) {
    InterpJob J{};
    J.y = y;
    J.ld = ld;
    J.n = g.n;
    J.m_in = p->iw.m_in;
    J.N = p->iw.N;
    J.in_f64 = p->d.in_dtype == CORR2D_DTYPE_F64;
    J.W = at<double>(ws, p->iw_off);
    J.range = (const int32_t*)(at<char>(ws, p->iw_off) + align256(p->iw.W.size() * sizeof(double)));
    J.out = at<double>(ws, out_off);
    J.ld_out = g.n_pad;
    hipError_t e = launch_interp(J, s);
    if (e != hipSuccess) return device_fail(e, "interpolation launch");
    return CORR2D_OK;
}

}  // namespace

corr2d_status corr2d_homo(corr2d_plan_t p, const void* y, const double* ref, void* phi, void* psi,
                          void* ws, size_t ws_bytes, void* stream) {
    if (!p) return fail(CORR2D_EINVAL, "NULL plan");
    if (p->batched) return fail(CORR2D_EINVAL, "batched plan passed to corr2d_homo");
    if (p->hetero) return fail(CORR2D_EINVAL, "heterocorrelation plan passed to corr2d_homo");
    if (!y || !phi || !psi) return fail(CORR2D_EINVAL, "NULL y, phi or psi");
    const size_t in_al = p->d.in_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    const size_t out_al = p->d.out_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    if (!aligned(y, in_al) || !aligned(phi, out_al) || !aligned(psi, out_al) || (ref && !aligned(ref, 8)))
        return fail(CORR2D_EINVAL, "misaligned data pointer");
    corr2d_status st = check_ws(p, ws, ws_bytes);
    if (st != CORR2D_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    TableSrcInline ts{};
    ts.j[0] = make_table_job(p, p->g1, ws, p->table_off);
    ts.count = 1;
    ts.blocks0 = table_blocks(p->g1);
    hipError_t e = merged_prep(p) ? hipSuccess : launch_prep_tables(p, ts, s);
    if (e != hipSuccess) return device_fail(e, "tables launch");

    const void* yc = y;
    int64_t ldc = p->d.ld_in1;
    if (p->interp) {
        st = upload_interp(p, ws, s);
        if (st == CORR2D_OK) st = resample(p, ws, y, p->d.ld_in1, p->g1, p->yi1_off, s);
        if (st != CORR2D_OK) return st;
        yc = at<char>(ws, p->yi1_off);
        ldc = p->g1.n_pad;
    }
    PrepSrcInline ps{};
    ps.j[0] = make_prep_job(p, p->g1, p->s1, yc, ldc, ref, ws, p->table_off);
    if (p->interp) ps.j[0].in_f64 = 1;
    ps.count = 1;
    ps.blocks0 = center_blocks(p->g1);
    // the FFT transform, and the fused table product, centre the spectra themselves
    if (merged_prep(p))
        e = launch_prep(ts, ts.blocks0, needs_qn(p) ? qn_blocks(p->g1.m) : 0, p->g1.m, ps,
                        p->fused_center ? 0 : ps.blocks0, s);
    else if (!p->fft && !p->fused_center)
        e = launch_center(ps, ps.blocks0, s);
    if (e != hipSuccess) return device_fail(e, "center launch");
    if (p->fft) {
        ps.blocks0 = fft_blocks(p->g1);
        e = launch_fft_transform(p->d.prec, fft_log2(p->g1.m), ps, ps.blocks0, s);
    } else {
        ps.blocks0 = prep_blocks(p->g1, p->d.prec, p->fused_center);
        e = p->fused_center ? launch_center_transform(p->d.prec, ps, ps.blocks0, s)
                            : launch_transform(p->d.prec, ps, ps.blocks0, s);
    }
    if (e != hipSuccess) return device_fail(e, "transform launch");
    if (p->rowsel && (e = launch_selection(p, ws, s)) != hipSuccess) return device_fail(e, "row selection launch");

    CorrJob C = make_corr_job(p, p->g1, p->s1, p->g1, p->s1, ws, phi, psi, true, p->c, p->tile,
                              p->d.ld_out, p->d.out_layout);
    if (p->rowsel) C.kb_sel = at<int32_t>(ws, p->sel_off);
    if (g_ev_before) (void)hipEventRecord(g_ev_before, s);
    e = launch_corr(p->d.prec, p->tile.fm, p->tile.fn, C, C.ntiles, s);
    if (e != hipSuccess) return device_fail(e, "correlation launch");
    if (g_ev_after) (void)hipEventRecord(g_ev_after, s);
    return ok();
}

corr2d_status corr2d_hetero(corr2d_plan_t p, const void* y1, const double* ref1, const void* y2,
                            const double* ref2, void* phi, void* psi, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!p) return fail(CORR2D_EINVAL, "NULL plan");
    if (p->batched || !p->hetero) return fail(CORR2D_EINVAL, "plan is not a heterocorrelation plan");
    if (!y1 || !y2 || !phi || !psi) return fail(CORR2D_EINVAL, "NULL y1, y2, phi or psi");
    const size_t in_al = p->d.in_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    const size_t out_al = p->d.out_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    if (!aligned(y1, in_al) || !aligned(y2, in_al) || !aligned(phi, out_al) || !aligned(psi, out_al) ||
        (ref1 && !aligned(ref1, 8)) || (ref2 && !aligned(ref2, 8)))
        return fail(CORR2D_EINVAL, "misaligned data pointer");
    corr2d_status st = check_ws(p, ws, ws_bytes);
    if (st != CORR2D_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    TableSrcInline ts{};
    ts.j[0] = make_table_job(p, p->g1, ws, p->table_off);
    ts.count = 1;
    ts.blocks0 = table_blocks(p->g1);
    hipError_t e = merged_prep(p) ? hipSuccess : launch_prep_tables(p, ts, s);
    if (e != hipSuccess) return device_fail(e, "tables launch");

    const void *yc1 = y1, *yc2 = y2;
    int64_t ldc1 = p->d.ld_in1, ldc2 = p->d.ld_in2;
    if (p->interp) {
        st = upload_interp(p, ws, s);
        if (st == CORR2D_OK) st = resample(p, ws, y1, p->d.ld_in1, p->g1, p->yi1_off, s);
        if (st == CORR2D_OK) st = resample(p, ws, y2, p->d.ld_in2, p->g2, p->yi2_off, s);
        if (st != CORR2D_OK) return st;
        yc1 = at<char>(ws, p->yi1_off);
        yc2 = at<char>(ws, p->yi2_off);
        ldc1 = p->g1.n_pad;
        ldc2 = p->g2.n_pad;
    }
    PrepSrcInline ps{};
    ps.j[0] = make_prep_job(p, p->g1, p->s1, yc1, ldc1, ref1, ws, p->table_off);
    ps.j[1] = make_prep_job(p, p->g2, p->s2, yc2, ldc2, ref2, ws, p->table_off);
    if (p->interp) ps.j[0].in_f64 = ps.j[1].in_f64 = 1;
    ps.count = 2;
    ps.blocks0 = center_blocks(p->g1);
    if (merged_prep(p))
        e = launch_prep(ts, ts.blocks0, needs_qn(p) ? qn_blocks(p->g1.m) : 0, p->g1.m, ps,
                        p->fused_center ? 0 : ps.blocks0 + center_blocks(p->g2), s);
    else if (!p->fft && !p->fused_center)
        e = launch_center(ps, ps.blocks0 + center_blocks(p->g2), s);
    if (e != hipSuccess) return device_fail(e, "center launch");
    if (p->fft) {
        ps.blocks0 = fft_blocks(p->g1);
        e = launch_fft_transform(p->d.prec, fft_log2(p->g1.m), ps, ps.blocks0 + fft_blocks(p->g2), s);
    } else {
        ps.blocks0 = prep_blocks(p->g1, p->d.prec, p->fused_center);
        const int nb = ps.blocks0 + prep_blocks(p->g2, p->d.prec, p->fused_center);
        e = p->fused_center ? launch_center_transform(p->d.prec, ps, nb, s) : launch_transform(p->d.prec, ps, nb, s);
    }
    if (e != hipSuccess) return device_fail(e, "transform launch");
    if (p->rowsel && (e = launch_selection(p, ws, s)) != hipSuccess) return device_fail(e, "row selection launch");

    CorrJob C = make_corr_job(p, p->g1, p->s1, p->g2, p->s2, ws, phi, psi, false, p->c, p->tile,
                              p->d.ld_out, CORR2D_LAYOUT_FULL);
    if (p->rowsel) C.kb_sel = at<int32_t>(ws, p->sel_off);
    if (g_ev_before) (void)hipEventRecord(g_ev_before, s);
    e = launch_corr(p->d.prec, p->tile.fm, p->tile.fn, C, C.ntiles, s);
    if (e != hipSuccess) return device_fail(e, "correlation launch");
    if (g_ev_after) (void)hipEventRecord(g_ev_after, s);
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Checks of the allocation-free entry point (noalloc.hip)
// ---------------------------------------------------------------------------
namespace corr2d {

corr2d_status noalloc_fail(corr2d_status s, const char* what) { return fail(s, "%s", what); }

corr2d_status noalloc_check(corr2d_plan_t p, size_t max_bytes) {
    if (!p) return fail(CORR2D_EINVAL, "NULL plan");
    if (p->batched || p->hetero)
        return fail(CORR2D_EINVAL, "corr2d_homo_noalloc takes a homocorrelation plan");
    if (p->interp)
        return fail(CORR2D_EUNSUPPORTED,
                    "corr2d_homo_noalloc: interpolation plans stage their weights in pinned memory; "
                    "use corr2d_homo");
    if (p->ws_bytes > max_bytes)
        return fail(CORR2D_EWORKSPACE,
                    "corr2d_homo_noalloc: the plan needs a workspace of %zu bytes, more than the %zu "
                    "bytes of the fixed scratch; use corr2d_homo with a workspace",
                    p->ws_bytes, max_bytes);
    return CORR2D_OK;
}

}  // namespace corr2d

// ---------------------------------------------------------------------------
// Batched path
// ---------------------------------------------------------------------------
namespace {

// Fill the pinned host blob with the job arrays for these pointers.
void fill_blob(corr2d_plan_s* p, const void* y_base, void* phi_base, void* psi_base, void* ws) {
    const size_t nd = p->distinct_m.size(), count = p->items.size();
    const BlobLayout L = blob_layout(nd, count);
    char* h = (char*)p->host_blob;
    std::memset(h, 0, L.total);
    TableJob* tj = (TableJob*)(h + L.tables);
    int32_t* ts = (int32_t*)(h + L.tstart);
    int32_t blk = 0;
    for (size_t q = 0; q < nd; ++q) {
        const Geo g = geometry(p->distinct_m[q], 1, p->d.prec);
        tj[q] = make_table_job(p, g, ws, p->table_of_m[q]);
        ts[q] = blk;
        blk += table_blocks(g);
    }
    ts[nd] = blk;
    int32_t* qs = (int32_t*)(h + L.qstart);
    int32_t qb = 0;
    for (size_t q = 0; q < nd; ++q) {
        qs[q] = qb;
        qb += qn_blocks(p->distinct_m[q]);
    }
    qs[nd] = qb;
    PrepJob* pj = (PrepJob*)(h + L.prep);
    int32_t* cs = (int32_t*)(h + L.cstart);
    int32_t* xs = (int32_t*)(h + L.xstart);
    CorrJob* cj = (CorrJob*)(h + L.corr);
    int64_t* tst = (int64_t*)(h + L.tilestart);
    const size_t isz = p->d.in_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    const size_t osz = p->d.out_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    int32_t cb = 0, xb = 0;
    int64_t tt = 0;
    for (size_t r = 0; r < count; ++r) {
        const auto& I = p->items[p->order[r]];
        // tile numbers restart at 0 for each group's persistent launch
        for (const auto& gr : p->groups)
            if ((int)r == gr.first) tt = 0;
        const void* y = (const char*)y_base + I.it.in_offset * isz;
        pj[r] = make_prep_job(p, I.g, I.s, y, I.it.ld_in, nullptr, ws, I.table_off);
        cs[r] = cb;
        cb += center_blocks(I.g);
        xs[r] = xb;
        xb += prep_blocks(I.g, p->d.prec, p->fused_center);
        void* ph = (char*)phi_base + I.it.out_offset * osz;
        void* ps = (char*)psi_base + I.it.out_offset * osz;
        cj[r] = make_corr_job(p, I.g, I.s, I.g, I.s, ws, ph, ps, true, I.c, I.tile, I.it.n,
                              p->d.out_layout);
        tst[r] = tt;
        tt += cj[r].ntiles;
    }
    cs[count] = cb;
    xs[count] = xb;
    tst[count] = tt;
}

corr2d_status enqueue_batched(corr2d_plan_s* p, void* ws, hipStream_t s) {
    const size_t nd = p->distinct_m.size(), count = p->items.size();
    const BlobLayout L = blob_layout(nd, count);
    char* dev = at<char>(ws, p->jobs_off);
    hipError_t e = hipMemcpyAsync(dev, p->host_blob, L.total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_fail(e, "job upload");
    const char* h = (const char*)p->host_blob;
    int* counter = at<int>(ws, p->counter_off);

    TableSrcArray ta{};
    ta.jobs = (const TableJob*)(dev + L.tables);
    ta.start = (const int32_t*)(dev + L.tstart);
    ta.qstart = (const int32_t*)(dev + L.qstart);
    ta.count = (int32_t)nd;
    ta.counter = counter;
    ta.ncounters = (int32_t)p->groups.size();
    const int64_t max_m = *std::max_element(p->distinct_m.begin(), p->distinct_m.end());
    e = launch_tables(ta, ((const int32_t*)(h + L.tstart))[nd], max_m, s);
    if (e == hipSuccess && needs_qn(p)) e = launch_tables_qn(ta, ((const int32_t*)(h + L.qstart))[nd], max_m, s);
    if (e != hipSuccess) return device_fail(e, "tables launch");

    PrepSrcArray pa{};
    pa.jobs = (const PrepJob*)(dev + L.prep);
    pa.count = (int32_t)count;
    if (!p->fused_center) {
        pa.start = (const int32_t*)(dev + L.cstart);
        e = launch_center(pa, ((const int32_t*)(h + L.cstart))[count], s);
        if (e != hipSuccess) return device_fail(e, "center launch");
    }
    pa.start = (const int32_t*)(dev + L.xstart);
    const int xb = ((const int32_t*)(h + L.xstart))[count];
    e = p->fused_center ? launch_center_transform(p->d.prec, pa, xb, s) : launch_transform(p->d.prec, pa, xb, s);
    if (e != hipSuccess) return device_fail(e, "transform launch");

    int dev_id = 0, cus = 0;
    (void)hipGetDevice(&dev_id);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess || cus <= 0)
        cus = 256;
    // one persistent launch per tile shape, each with its own ticket counter
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        const auto& gr = p->groups[gi];
        const bool out_f64 = p->d.out_dtype == CORR2D_DTYPE_F64;
        const int per_cu = persistent_blocks_per_cu(p->d.prec, gr.tile.fm, gr.tile.fn, out_f64);
        int64_t blocks = (int64_t)cus * per_cu;
        blocks = std::min<int64_t>(blocks, gr.tiles);
        e = launch_corr_persistent(p->d.prec, gr.tile.fm, gr.tile.fn, out_f64,
                                   (const CorrJob*)(dev + L.corr) + gr.first,
                                   (const int64_t*)(dev + L.tilestart) + gr.first, gr.count, gr.tiles,
                                   counter + gi, (int)blocks, s);
        if (e != hipSuccess) return device_fail(e, "persistent correlation launch");
    }
    return CORR2D_OK;
}

corr2d_status enqueue_sequential(corr2d_plan_s* p, const void* y_base, void* phi_base,
                                 void* psi_base, void* ws, hipStream_t s) {
    const size_t isz = p->d.in_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    const size_t osz = p->d.out_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    for (size_t r = 0; r < p->items.size(); ++r) {
        const auto& I = p->items[r];
        TableSrcInline ts{};
        ts.j[0] = make_table_job(p, I.g, ws, I.table_off);
        ts.count = 1;
        ts.blocks0 = table_blocks(I.g);
        hipError_t e = launch_tables(ts, ts.blocks0, I.g.m, s);
        if (e == hipSuccess && needs_qn(p)) e = launch_tables_qn(ts, qn_blocks(I.g.m), I.g.m, s);
        if (e != hipSuccess) return device_fail(e, "tables launch");
        PrepSrcInline ps{};
        ps.j[0] = make_prep_job(p, I.g, I.s, (const char*)y_base + I.it.in_offset * isz, I.it.ld_in,
                                nullptr, ws, I.table_off);
        ps.count = 1;
        ps.blocks0 = center_blocks(I.g);
        if (!p->fused_center) e = launch_center(ps, ps.blocks0, s);
        if (e != hipSuccess) return device_fail(e, "center launch");
        ps.blocks0 = prep_blocks(I.g, p->d.prec, p->fused_center);
        e = p->fused_center ? launch_center_transform(p->d.prec, ps, ps.blocks0, s)
                            : launch_transform(p->d.prec, ps, ps.blocks0, s);
        if (e != hipSuccess) return device_fail(e, "transform launch");
        CorrJob C = make_corr_job(p, I.g, I.s, I.g, I.s, ws, (char*)phi_base + I.it.out_offset * osz,
                                  (char*)psi_base + I.it.out_offset * osz, true, I.c, I.tile, I.it.n,
                                  p->d.out_layout);
        e = launch_corr(p->d.prec, I.tile.fm, I.tile.fn, C, C.ntiles, s);
        if (e != hipSuccess) return device_fail(e, "correlation launch");
    }
    return CORR2D_OK;
}

// Mark the pinned job buffer as read by the work just enqueued on s.
corr2d_status record_blob_use(corr2d_plan_s* p, hipStream_t s) {
    hipError_t e = hipEventRecord(p->blob_done, s);
    if (e != hipSuccess) return device_fail(e, "event record");
    p->blob_recorded = true;
    return ok();
}

}  // namespace

extern "C" corr2d_status corr2d_batched(corr2d_plan_t p, const void* y_base, void* phi_base,
                                        void* psi_base, void* ws, size_t ws_bytes, void* stream) {
    if (!p) return fail(CORR2D_EINVAL, "NULL plan");
    if (!p->batched) return fail(CORR2D_EINVAL, "plan is not a batched plan");
    if (!y_base || !phi_base || !psi_base) return fail(CORR2D_EINVAL, "NULL base pointer");
    const size_t in_al = p->d.in_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    const size_t out_al = p->d.out_dtype == CORR2D_DTYPE_F64 ? 8 : 4;
    if (!aligned(y_base, in_al) || !aligned(phi_base, out_al) || !aligned(psi_base, out_al))
        return fail(CORR2D_EINVAL, "misaligned data pointer");
    corr2d_status st = check_ws(p, ws, ws_bytes);
    if (st != CORR2D_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(p->mu);

    if (p->d.flags & CORR2D_FLAG_SEQUENTIAL) {
        st = enqueue_sequential(p, y_base, phi_base, psi_base, ws, s);
        return st == CORR2D_OK ? ok() : st;
    }

    corr2d_plan_s::GraphKey key;
    key.y = y_base;
    key.phi = phi_base;
    key.psi = psi_base;
    key.ws = ws;
    key.stream = stream;
    const BlobLayout L = blob_layout(p->distinct_m.size(), p->items.size());
    if (!p->host_blob) {
        hipError_t e = hipHostMalloc(&p->host_blob, L.total, hipHostMallocDefault);
        if (e != hipSuccess) { p->host_blob = nullptr; return device_fail(e, "pinned job buffer"); }
    }
    if (!p->blob_done) {
        hipError_t e = hipEventCreateWithFlags(&p->blob_done, hipEventDisableTiming);
        if (e != hipSuccess) { p->blob_done = nullptr; return device_fail(e, "event creation"); }
    }
    if (!p->blob_valid || !(p->blob_key == key)) {
        // the previous blob may still be read by an enqueued copy: wait for
        // the last call that used it (that call's stream only)
        if (p->blob_recorded) {
            hipError_t e = hipEventSynchronize(p->blob_done);
            if (e != hipSuccess) return device_fail(e, "wait for the previous job upload");
        }
        fill_blob(p, y_base, phi_base, psi_base, ws);
        p->blob_valid = true;
        p->blob_key = key;
        if (p->have_graph) {
            (void)hipGraphExecDestroy(p->gexec);
            p->gexec = nullptr;
            p->have_graph = false;
        }
    }

    if (p->d.flags & CORR2D_FLAG_NO_GRAPH) {
        st = enqueue_batched(p, ws, s);
        if (st != CORR2D_OK) return st;
        return record_blob_use(p, s);
    }
    if (!p->have_graph) {
        hipStream_t cs = s;
        bool own = false;
        if (cs == nullptr) {
            // the legacy default stream cannot be captured: capture on a private stream
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
                return fail(CORR2D_EDEVICE, "stream creation for graph capture failed");
            own = true;
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            if (own) (void)hipStreamDestroy(cs);
            return device_fail(e, "begin capture");
        }
        corr2d_status est = enqueue_batched(p, ws, cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (own) (void)hipStreamDestroy(cs);
        if (est != CORR2D_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return est;
        }
        if (e != hipSuccess) return device_fail(e, "end capture");
        e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return device_fail(e, "graph instantiate");
        p->have_graph = true;
    }
    hipError_t e = hipGraphLaunch(p->gexec, s);
    if (e != hipSuccess) return device_fail(e, "graph launch");
    return record_blob_use(p, s);
}
