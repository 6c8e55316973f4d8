"""The operator's tile order on a box mesh (walk.h): host-side checks of the very
header the kernels include, compiled with the host compiler.  Every walk must be
a permutation of the tiles (each tile visited once, none out of range), the
identity where tiles would straddle rows (padded rows: every element in exactly
one tile, every tile in one row), and it must bring z-neighbours within one slab
plane (the locality it exists for)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2202_12477_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "walk.h"
using namespace hb;
static int check(int nx, int ny, int nz, int epb) {
    const TileWalk w = make_walk(nx, ny, nz, epb);
    const long E = (long)nx * ny * nz;
    if (nx % epb != 0) {
        if (w.txn != 0) return 1;
        for (uint32_t j = 0; j < 64 && j < E; ++j) if (walk_tile(w, j) != j) return 2;
        return 0;
    }
    const long T = E / epb;
    if ((long)w.txn * w.ny * w.nz != T) return 3;
    std::vector<int> seen(T, 0);
    for (long j = 0; j < T; ++j) {
        const uint32_t t = walk_tile(w, (uint32_t)j);
        if ((long)t >= T) return 4;
        if (seen[t]++) return 5;
    }
    return 0;
}
// padded rows: ceil(nx/epb) tiles per row; the spans of the walk's tiles cover
// every element exactly once, each inside one row, the short one last in its row
static int check_padded(int nx, int ny, int nz, int epb) {
    const TileWalk w = make_walk(nx, ny, nz, epb, true);
    const long E = (long)nx * ny * nz;
    const long tpr = (nx + epb - 1) / epb, T = tpr * ny * nz;
    if (walk_tiles(w, E, epb) != T || (long)w.txn != tpr) return 11;
    if ((nx % epb == 0) != (w.rowlen == 0)) return 12;
    std::vector<int> seen(E, 0), tseen(T, 0);
    for (long j = 0; j < T; ++j) {
        const uint32_t t = walk_tile(w, (uint32_t)j);
        if ((long)t >= T || tseen[t]++) return 13;
        const TileSpan sp = tile_span(w, t, E, epb);
        if (sp.n < 1 || sp.n > epb || sp.e0 < 0 || sp.e0 + sp.n > E) return 14;
        if (sp.e0 / nx != (sp.e0 + sp.n - 1) / nx) return 15;          // one row
        if (sp.n < epb && (sp.e0 + sp.n) % nx != 0) return 16;          // short tiles end their row
        for (int k = 0; k < sp.n; ++k) if (seen[sp.e0 + k]++) return 17;
    }
    for (long e = 0; e < E; ++e) if (seen[e] != 1) return 18;
    return 0;
}
int main() {
    int bad = 0, n = 0;
    for (int nx = 1; nx <= 13; ++nx)
        for (int ny = 1; ny <= 11; ++ny)
            for (int nz = 1; nz <= 3; ++nz)
                for (int epb = 1; epb <= 5; ++epb) { int r = check_padded(nx, ny, nz, epb); ++n; if (r) { ++bad; std::printf("bad padded %d %d %d %d: %d\n", nx, ny, nz, epb, r); } }
    { int r = check_padded(50, 50, 50, 4); ++n; if (r) { ++bad; std::printf("bad padded 50^3: %d\n", r); } }
    for (int nx = 1; nx <= 13; ++nx)
        for (int ny = 1; ny <= 19; ++ny)
            for (int nz = 1; nz <= 5; ++nz)
                for (int epb = 1; epb <= 5; ++epb) { int r = check(nx, ny, nz, epb); ++n; if (r) { ++bad; std::printf("bad %d %d %d %d: %d\n", nx, ny, nz, epb, r); } }
    const int big[][4] = {{32, 32, 32, 1}, {32, 32, 32, 4}, {21, 21, 21, 1}, {26, 26, 26, 2}, {28, 28, 28, 3},
                          {64, 64, 64, 16}, {128, 128, 128, 64}, {16, 16, 16, 1}, {40, 9, 33, 8}};
    for (auto &b : big) { int r = check(b[0], b[1], b[2], b[3]); ++n; if (r) { ++bad; std::printf("bad %d %d %d %d: %d\n", b[0], b[1], b[2], b[3], r); } }
    // locality on the 32^3 box, one element per tile: y-neighbours one row
    // (32 tiles) and z-neighbours one slab plane (32 * 4 tiles) later in the walk
    const TileWalk w = make_walk(32, 32, 32, 1);
    std::vector<long> pos(32768);
    for (long j = 0; j < 32768; ++j) pos[walk_tile(w, (uint32_t)j)] = j;
    long dy = 0, dz = 0;
    for (int z = 0; z < 32; ++z) for (int y = 0; y < 32; ++y) for (int x = 0; x < 32; ++x) {
        const long t = x + 32 * (y + 32 * z);
        if (y % 4 != 3 && y + 1 < 32) dy = std::max(dy, std::labs(pos[t + 32] - pos[t]));
        if (z + 1 < 32) dz = std::max(dz, std::labs(pos[t + 1024] - pos[t]));
    }
    std::printf("checked %d walks, %d bad, dy %ld dz %ld\n", n, bad, dy, dz);
    return bad != 0 || dy != 32 || dz != 128;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_walk_is_a_permutation_of_the_tiles():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "walk_check.cpp"), os.path.join(d, "walk_check")
        with open(src, "w") as f:
            f.write(HARNESS.replace("#include <vector>", "#include <vector>\n#include <algorithm>\n#include <cstdlib>"))
        subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(out.stdout)
        assert out.returncode == 0, out.stdout[-2000:]
        assert "0 bad" in out.stdout
