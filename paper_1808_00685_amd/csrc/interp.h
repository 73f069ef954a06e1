// interp.h -- interpolation weights of a plan (host side).
#pragma once
#include <stdint.h>

#include <vector>

#include "corr2d_internal.h"

namespace corr2d {

struct InterpWeights {
    int64_t m_in = 0, N = 0;
    std::vector<double> W;               // N x m_in, row-major
    std::vector<int32_t> block_range;    // per block of kInterpRows output rows: [lo, hi)
};

// method 1: piecewise linear, 2: FMM cubic spline.  t_in strictly increasing.
// Returns false if a weight is not finite.
bool build_interp_weights(const double* t_in, int64_t m_in, int64_t N, int method, InterpWeights& w);

}  // namespace corr2d
