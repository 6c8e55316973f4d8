// The order in which an operator launch visits the tiles of a box mesh.
//
// A tile is `epb` consecutive elements of one x-row of the box (when epb divides
// nx), so the tiles form a txn x ny x nz grid (txn = nx/epb) numbered like the
// elements, x fastest.  The walk cuts the box into slabs of `ys` element rows in
// y and visits the slabs one after the other; inside a slab it visits the
// z-planes in order, each plane's rows, each row's tiles.  An operator launch
// hands every XCD a contiguous range of the walk, so an element meets its
// y-neighbours txn tiles later and its z-neighbours txn*ys tiles later: with a
// slab per XCD (ys = ny/8), both are inside the set of tiles the XCD has in
// flight, and the lines of x and y that neighbouring elements share are still in
// that XCD's L2 when the second element reaches them.  (In plain element order a
// z-neighbour comes nx*ny elements later, after the lines have been evicted and
// written back: the written bytes of y doubled.)
//
// Plain constexpr arithmetic, so host code (list building, tests) and device
// code evaluate the same function.
#pragma once

#include <cstdint>

namespace hb {

struct TileWalk {
    uint32_t txn = 0, ny = 0, nz = 0, ys = 0;  // txn == 0: identity (plain element order)
};

// The j-th tile of the walk, 0 <= j < txn*ny*nz.
constexpr uint32_t walk_tile(const TileWalk &w, uint32_t j)
{
    if (w.txn == 0) return j;
    const uint32_t slab = w.txn * w.ys * w.nz;  // tiles in a full slab
    const uint32_t s = j / slab;
    const uint32_t y0 = s * w.ys;
    const uint32_t h = w.ny - y0 < w.ys ? w.ny - y0 : w.ys;  // rows of this slab (the last may be short)
    const uint32_t r = j - s * slab;
    const uint32_t plane = w.txn * h;
    const uint32_t z = r / plane;
    const uint32_t r2 = r - z * plane;
    const uint32_t yy = r2 / w.txn;
    const uint32_t x = r2 - yy * w.txn;
    return x + w.txn * (y0 + yy + w.ny * z);
}

// The walk for a box of nx x ny x nz elements cut into tiles of epb elements;
// identity where a tile would straddle two rows.
constexpr TileWalk make_walk(int64_t nx, int64_t ny, int64_t nz, int epb)
{
    TileWalk w;
    if (epb < 1 || nx % epb != 0) return w;
    w.txn = static_cast<uint32_t>(nx / epb);
    w.ny = static_cast<uint32_t>(ny);
    w.nz = static_cast<uint32_t>(nz);
    w.ys = static_cast<uint32_t>((ny + 7) / 8);  // one slab per XCD
    return w;
}

}  // namespace hb
