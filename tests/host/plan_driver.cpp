// plan_driver.cpp -- exercises the host-side plan code of the C ABI under
// address and undefined-behaviour sanitizers, without a GPU: descriptor
// defaults, plan validation over valid and invalid descriptors, plans with
// interpolation weights, heterocorrelation and batched plans, plan info and
// workspace sizes, status strings, and compute calls whose arguments fail
// validation before any device work.  Exit status 0 when every expectation
// holds; each failed expectation is printed.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "corr2d.h"

static int g_fail = 0;
#define EXPECT(c)                                                            \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n",    \
                         __FILE__, __LINE__, #c, corr2d_last_error());       \
            ++g_fail;                                                        \
        }                                                                    \
    } while (0)

static corr2d_status try_plan(const corr2d_desc& d, corr2d_plan_info* info = nullptr) {
    corr2d_plan_t p = nullptr;
    const corr2d_status s = corr2d_plan(&p, &d);
    if (s == CORR2D_OK) {
        EXPECT(p != nullptr);
        size_t ws = 0;
        EXPECT(corr2d_workspace_bytes(p, &ws) == CORR2D_OK && ws % 256 == 0);
        corr2d_plan_info pi;
        EXPECT(corr2d_plan_get_info(p, &pi) == CORR2D_OK && pi.workspace_bytes == ws);
        if (info) *info = pi;
        EXPECT(corr2d_plan_destroy(p) == CORR2D_OK);
    } else {
        EXPECT(p == nullptr);
    }
    return s;
}

int main() {
    corr2d_desc d;
    corr2d_desc_init(&d);
    EXPECT(d.prec == CORR2D_PREC_SPLIT_BF16 && d.out_layout == CORR2D_LAYOUT_FULL);

    // every precision x layout x basis x kernel over a range of sizes
    const int64_t ms[] = {2, 3, 11, 64, 127, 128, 256, 300, 1024, 4096};
    const int64_t ns[] = {1, 7, 129, 4096, 16384};
    int ok = 0;
    for (int prec = 0; prec <= 6; ++prec)
        for (int layout = 0; layout <= 2; ++layout)
            for (int basis = 0; basis <= 2; ++basis)
                for (int hil = 0; hil <= 2; ++hil)
                    for (int64_t m : ms)
                        for (int64_t n : ns) {
                            corr2d_desc_init(&d);
                            d.m = m;
                            d.n1 = n;
                            d.prec = prec;
                            d.out_layout = layout;
                            d.basis = basis;
                            d.hilbert = hil;
                            corr2d_plan_info info;
                            const corr2d_status s = try_plan(d, &info);
                            if (basis == CORR2D_BASIS_TIME && hil == CORR2D_HILBERT_R_COMPAT) {
                                EXPECT(s == CORR2D_EUNSUPPORTED);
                                continue;
                            }
                            EXPECT(s == CORR2D_OK);
                            if (s != CORR2D_OK) continue;
                            ++ok;
                            EXPECT(info.n_pad >= n && info.k_pad >= m && info.tiles > 0);
                            const bool pow2 = (m & (m - 1)) == 0 && m >= 128 && m <= 1024;
                            EXPECT(basis == CORR2D_BASIS_AUTO ? info.basis <= 1 : info.basis == basis);
                            const bool fft = pow2 && (info.basis == CORR2D_BASIS_FOURIER || hil == CORR2D_HILBERT_NODA);
                            EXPECT(info.transform == (fft ? 1 : 0));
                        }
    EXPECT(ok > 1000);

    // row-selective split: split formats, Fourier basis, m <= 1024
    for (int prec : {CORR2D_PREC_SPLIT_BF16, CORR2D_PREC_SPLIT_F16, CORR2D_PREC_F32})
        for (int64_t m : ms)
            for (int64_t n2 : {(int64_t)0, (int64_t)300}) {
                corr2d_desc_init(&d);
                d.m = m;
                d.n1 = 4096;
                d.n2 = n2;
                d.prec = prec;
                d.flags = CORR2D_FLAG_SPLIT_ROWS;
                d.split_tol = 1e-4;
                corr2d_plan_info info;
                const corr2d_status s = try_plan(d, &info);
                if (prec == CORR2D_PREC_F32 || m > 1024) {
                    EXPECT(s == CORR2D_EUNSUPPORTED);
                    continue;
                }
                EXPECT(s == CORR2D_OK);
                EXPECT(info.sel_offset > 0 && info.sel_offset + 65 * 4 <= info.workspace_bytes);
            }

    // heterocorrelation, strides, result scaling, flags
    corr2d_desc_init(&d);
    d.m = 128; d.n1 = 8192; d.n2 = 2048; d.prec = CORR2D_PREC_F16; d.ld_in1 = 9000; d.ld_out = 3000;
    d.scale_alpha = 0.5;
    EXPECT(try_plan(d) == CORR2D_OK);
    d.out_layout = CORR2D_LAYOUT_UPPER_PACKED;
    EXPECT(try_plan(d) == CORR2D_EINVAL);
    corr2d_desc_init(&d);
    d.m = 256; d.n1 = 1000; d.flags = CORR2D_FLAG_TRANSFORM_MATMUL;
    corr2d_plan_info info;
    EXPECT(try_plan(d, &info) == CORR2D_OK && info.transform == 0);
    d.flags = 0x40;
    EXPECT(try_plan(d) == CORR2D_EINVAL);

    // invalid descriptors
    struct Bad { int64_t m, n1, n2, ld1; int prec, layout; double alpha; corr2d_status want; };
    const Bad bad[] = {{1, 10, 0, 0, 2, 0, 0.0, CORR2D_EINVAL},
                       {4, 0, 0, 0, 2, 0, 0.0, CORR2D_EINVAL},
                       {4, 10, -1, 0, 2, 0, 0.0, CORR2D_EINVAL},
                       {4, 10, 0, 5, 2, 0, 0.0, CORR2D_EINVAL},
                       {4, 10, 0, 0, 9, 0, 0.0, CORR2D_EINVAL},
                       {4, 10, 0, 0, 2, 7, 0.0, CORR2D_EINVAL},
                       {4, 10, 0, 0, 2, 0, NAN, CORR2D_EINVAL},
                       {5000, 10, 0, 0, 2, 0, 0.0, CORR2D_EUNSUPPORTED},
                       {4, (int64_t)1 << 25, 0, 0, 2, 0, 0.0, CORR2D_EINVAL}};
    for (const Bad& b : bad) {
        corr2d_desc_init(&d);
        d.m = b.m; d.n1 = b.n1; d.n2 = b.n2; d.ld_in1 = b.ld1; d.prec = b.prec; d.out_layout = b.layout;
        d.scale_alpha = b.alpha;
        EXPECT(try_plan(d) == b.want);
        EXPECT(std::strlen(corr2d_last_error()) > 0);
    }

    // interpolation weights (built on the host with the plan)
    for (int method = 1; method <= 2; ++method)
        for (int m_in : {2, 3, 4, 9, 70}) {
            std::vector<double> t(m_in);
            for (int i = 0; i < m_in; ++i) t[i] = 0.5 * i + 0.3 * std::sin(1.7 * i) * (i > 0);
            for (int i = 1; i < m_in; ++i)
                if (!(t[i] > t[i - 1])) t[i] = t[i - 1] + 0.1;
            for (int64_t m_out : {2, 33, 128, 400}) {
                corr2d_desc_init(&d);
                d.m = m_out; d.n1 = 300; d.interp = method; d.t_in = t.data(); d.m_in = m_in;
                EXPECT(try_plan(d) == CORR2D_OK);
                d.n2 = 77;
                EXPECT(try_plan(d) == CORR2D_OK);
            }
        }
    std::vector<double> tbad = {0.0, 1.0, 1.0, 2.0};
    corr2d_desc_init(&d);
    d.m = 8; d.n1 = 10; d.interp = CORR2D_INTERP_SPLINE; d.t_in = tbad.data(); d.m_in = 4;
    EXPECT(try_plan(d) == CORR2D_EINVAL);

    // batched plans
    std::vector<corr2d_item> items;
    int64_t out = 0;
    for (int i = 0; i < 64; ++i) {
        corr2d_item it;
        std::memset(&it, 0, sizeof it);
        it.m = 8 + (i * 37) % 193;
        it.n = 256 + (i * 977) % 7937;
        it.in_offset = 0;
        it.out_offset = out;
        out += it.n * it.n;
        items.push_back(it);
    }
    for (int prec : {CORR2D_PREC_F32, CORR2D_PREC_SPLIT_BF16, CORR2D_PREC_F64}) {
        corr2d_desc_init(&d);
        d.prec = prec;
        corr2d_plan_t p = nullptr;
        EXPECT(corr2d_batched_plan(&p, &d, items.data(), (int64_t)items.size()) == CORR2D_OK);
        corr2d_plan_info pi;
        EXPECT(corr2d_plan_get_info(p, &pi) == CORR2D_OK && pi.items == 64 && pi.out_elements == out);
        EXPECT(corr2d_plan_destroy(p) == CORR2D_OK);
    }
    items[3].m = 1;
    corr2d_plan_t pb = nullptr;
    EXPECT(corr2d_batched_plan(&pb, &d, items.data(), (int64_t)items.size()) == CORR2D_EINVAL && pb == nullptr);

    // compute calls that fail validation before any device work
    corr2d_desc_init(&d);
    d.m = 11; d.n1 = 64;
    corr2d_plan_t p = nullptr;
    EXPECT(corr2d_plan(&p, &d) == CORR2D_OK);
    size_t need = 0;
    corr2d_workspace_bytes(p, &need);
    alignas(256) static char fake_ws[256];
    double* fake = reinterpret_cast<double*>(fake_ws);
    EXPECT(corr2d_homo(p, nullptr, nullptr, fake, fake, fake_ws, need, nullptr) == CORR2D_EINVAL);
    EXPECT(corr2d_homo(p, fake_ws + 1, nullptr, fake, fake, fake_ws, need, nullptr) == CORR2D_EINVAL);
    EXPECT(corr2d_homo(p, fake, nullptr, fake, fake, fake_ws, need - 256, nullptr) == CORR2D_EWORKSPACE);
    EXPECT(corr2d_homo(p, fake, nullptr, fake, fake, nullptr, need, nullptr) == CORR2D_EWORKSPACE);
    EXPECT(corr2d_hetero(p, fake, nullptr, fake, nullptr, fake, fake, fake_ws, need, nullptr) == CORR2D_EINVAL);
    EXPECT(corr2d_batched(p, fake, fake, fake, fake_ws, need, nullptr) == CORR2D_EINVAL);
    EXPECT(corr2d_plan_destroy(p) == CORR2D_OK);
    EXPECT(corr2d_plan_destroy(nullptr) == CORR2D_OK);   // NULL is accepted

    for (int s = 0; s <= 5; ++s) EXPECT(std::strlen(corr2d_status_str((corr2d_status)s)) > 0);
    EXPECT(std::strlen(corr2d_version()) > 0);
    if (g_fail == 0) std::printf("plan driver: all expectations hold (%d plans over the grid)\n", ok);
    return g_fail == 0 ? 0 : 1;
}
