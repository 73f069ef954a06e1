// tune.h -- tile choice from the autotuned table.
#pragma once
#include <stdint.h>

namespace corr2d {
// Tile id (1: 64x64 output tiles, 2: 128x128) for a precision and problem
// size.  Reads the table named by CORR2D_TUNE_TABLE, else tune/gfx950.tsv
// next to the library; without a table a size rule is used.
int tune_lookup(int prec, int64_t m, int64_t n);
// Where the rules came from (the table's path and rule count, or the size
// rule), for the plan log.
const char* tune_source();
}
