// tile_order.h -- order in which the contraction kernels visit output tiles.
//
// Consecutive tile numbers run at the same time on the CUs of one XCD (the
// kernels remap workgroup ids so that each XCD takes a contiguous range), so
// the order decides which operand panels share an L2: tiles are grouped by G
// column tiles, and inside a group the row tiles follow one another, each
// taking the group's columns.  Both decoders are O(1) in the tile number.
#ifndef CORR2D_TILE_ORDER_H
#define CORR2D_TILE_ORDER_H

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace corr2d {

// Upper triangle for row tiles R times as tall as the column tiles are wide:
// row tile I covers rows [I R w, (I+1) R w) for column tiles of width w, so
// tile (I, J) holds an element with j >= i exactly when J >= R I.
// Tiles in the column tiles [0, x): the sum over J < x of floor(J/R) + 1.
__host__ __device__ inline int64_t upper_tiles_before(int64_t x, int R) {
    const int64_t q = x / R, r = x % R;
    return x + R * q * (q - 1) / 2 + r * q;
}

// Tile number t (0 <= t < R TI (TI+1) / 2, TJ = R TI) -> (I, J).  Group g
// covers the column tiles [gG, gG+G); its first tile is number
// upper_tiles_before(gG), about (gG)^2 / (2R), so g comes from a square root
// and an exact integer correction.  Inside the group, the rows whose first
// tile lies left of the group (I <= gG/R) take all its columns; the rows
// below take the columns from R I on.
__host__ __device__ inline void decode_upper(int64_t t, int TI, int TJ, int R, int G, int& I, int& J) {
    const int ng = (TJ + G - 1) / G;
    int g = (int)(sqrt(2.0 * R * (double)t) / G);
    g = g < ng - 1 ? g : ng - 1;
    while (g > 0 && upper_tiles_before((int64_t)g * G, R) > t) --g;
    while (g + 1 < ng && upper_tiles_before((int64_t)(g + 1) * G, R) <= t) ++g;
    const int c0 = g * G, c1 = c0 + G < TJ ? c0 + G : TJ;
    t -= upper_tiles_before(c0, R);
    const int nfull = c0 / R + 1 < TI ? c0 / R + 1 : TI;
    const int gw = c1 - c0;
    if (t < (int64_t)nfull * gw) {
        I = (int)(t / gw);
        J = c0 + (int)(t % gw);
        return;
    }
    t -= (int64_t)nfull * gw;
    int r = nfull;
    while (t >= c1 - R * r) { t -= c1 - R * r; ++r; }
    I = r;
    J = R * r + (int)t;
}

// Full Ti x Tj grid (heterocorrelation), grouped the same way.
__host__ __device__ inline void decode_full(int64_t t, int Ti, int Tj, int G, int& I, int& J) {
    const int64_t per_group = (int64_t)Ti * G;
    const int g = (int)(t / per_group);
    const int64_t r = t - (int64_t)g * per_group;
    const int gw = G < Tj - g * G ? G : Tj - g * G;
    I = (int)(r / gw);
    J = g * G + (int)(r % gw);
}

}  // namespace corr2d

#endif
