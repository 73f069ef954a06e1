"""The contraction's tile order (csrc/tile_order.h), built for the host.

decode_upper finds a tile's column group from a square root and an integer
correction; these tests compare it, and decode_full, tile by tile with the
order written as plain nested loops, over grids up to millions of tiles.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_00685_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROG = r'''
#include "tile_order.h"
#include <cstdio>
#include <cstdlib>
#include <vector>
// Reference orders as nested loops: column groups of G tiles; in a group the
// row tiles top to bottom, each row's tiles of the group left to right
// (upper triangle: from column tile R I on).
int main(int argc, char** argv) {
    const int TI = atoi(argv[1]), R = atoi(argv[2]), G = atoi(argv[3]);
    const int Ti = atoi(argv[4]), Tj = atoi(argv[5]);
    const int TJ = R * TI;
    long long t = 0, bad = 0;
    for (int c0 = 0; c0 < TJ; c0 += G)
        for (int I = 0; I < TI; ++I)
            for (int J = (c0 > R * I ? c0 : R * I); J < (c0 + G < TJ ? c0 + G : TJ); ++J, ++t) {
                int i, j;
                corr2d::decode_upper(t, TI, TJ, R, G, i, j);
                if (i != I || j != J) { if (!bad) printf("upper t=%lld got (%d,%d) want (%d,%d)\n", t, i, j, I, J); ++bad; }
            }
    const long long nu = t;
    t = 0;
    for (int c0 = 0; c0 < Tj; c0 += G)
        for (int I = 0; I < Ti; ++I)
            for (int J = c0; J < (c0 + G < Tj ? c0 + G : Tj); ++J, ++t) {
                int i, j;
                corr2d::decode_full(t, Ti, Tj, G, i, j);
                if (i != I || j != J) { if (!bad) printf("full t=%lld got (%d,%d) want (%d,%d)\n", t, i, j, I, J); ++bad; }
            }
    printf("%lld %lld %lld\n", nu, t, bad);
    return 0;
}
'''


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    d = tmp_path_factory.mktemp("tile_order")
    src = d / "t.hip"
    src.write_text(PROG)
    exe = d / "t"
    r = subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-I" + CSRC, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


@pytest.mark.parametrize("TI,R,G,Ti,Tj", [
    (1, 1, 8, 1, 1), (4, 1, 2, 3, 5), (5, 1, 8, 7, 9), (128, 1, 8, 64, 16), (64, 2, 8, 128, 128),
    (33, 2, 8, 33, 17), (7, 2, 3, 7, 10), (100, 1, 1, 10, 10), (16, 1, 32, 5, 70), (9, 3, 4, 2, 3),
    (2000, 1, 8, 1000, 999), (1500, 2, 8, 3, 3000),
])
def test_decoders_follow_the_loop_order(prog, TI, R, G, Ti, Tj):
    out = subprocess.run([prog, str(TI), str(R), str(G), str(Ti), str(Tj)], capture_output=True,
                         text=True, timeout=120).stdout.split()
    nu, nf, bad = (int(x) for x in out[-3:])
    assert bad == 0, " ".join(out[:-3])
    assert nu == R * TI * (TI + 1) // 2      # the count the plan launches
    assert nf == Ti * Tj
