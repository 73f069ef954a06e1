// launch_stubs.cpp -- link-time stand-ins for the kernel launchers of
// kernels.hip, so that the host-side plan code (api.cpp, tune.cpp,
// interp.cpp) can be built with address and undefined-behaviour sanitizers
// and exercised on a machine without a GPU.  The driver never reaches a
// launch: every call it makes fails validation first, and each stub aborts
// if it is reached anyway.
#include <cstdio>
#include <cstdlib>

#include "launch.h"

namespace corr2d {
namespace {
[[noreturn]] void reached(const char* what) {
    std::fprintf(stderr, "launch stub reached: %s\n", what);
    std::abort();
}
}  // namespace

hipError_t launch_tables(const TableSrcInline&, int, int64_t, hipStream_t) { reached("tables"); }
hipError_t launch_tables(const TableSrcArray&, int, int64_t, hipStream_t) { reached("tables"); }
hipError_t launch_tables_qn(const TableSrcInline&, int, int64_t, hipStream_t) { reached("tables_qn"); }
hipError_t launch_tables_qn(const TableSrcArray&, int, int64_t, hipStream_t) { reached("tables_qn"); }
hipError_t launch_center(const PrepSrcInline&, int, hipStream_t) { reached("center"); }
hipError_t launch_center(const PrepSrcArray&, int, hipStream_t) { reached("center"); }
hipError_t launch_prep(const TableSrcInline&, int, int, int64_t, const PrepSrcInline&, int, hipStream_t) {
    reached("prep");
}
hipError_t launch_transform(int, const PrepSrcInline&, int, hipStream_t) { reached("transform"); }
hipError_t launch_transform(int, const PrepSrcArray&, int, hipStream_t) { reached("transform"); }
hipError_t launch_center_transform(int, const PrepSrcInline&, int, hipStream_t) { reached("center_transform"); }
hipError_t launch_center_transform(int, const PrepSrcArray&, int, hipStream_t) { reached("center_transform"); }
hipError_t launch_fft_tables(const TableSrcInline&, int64_t, hipStream_t) { reached("fft_tables"); }
hipError_t launch_fft_transform(int, int, const PrepSrcInline&, int, hipStream_t) { reached("fft_transform"); }
hipError_t launch_corr(int, int, int, const CorrJob&, int64_t, hipStream_t) { reached("corr"); }
hipError_t launch_corr_persistent(int, int, int, bool, const CorrJob*, const int64_t*, int, int64_t, int*, int,
                                  hipStream_t) {
    reached("corr_persistent");
}
hipError_t launch_interp(const InterpJob&, hipStream_t) { reached("interp"); }
hipError_t launch_row_select(const SelJob&, hipStream_t) { reached("row_select"); }
// Every tile and precision pair that passes plan validation is built.
int corr_variant_supported(int, int, int) { return 1; }
int persistent_blocks_per_cu(int, int, int, bool) { reached("persistent_blocks_per_cu"); }
}  // namespace corr2d
