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
// With padded rows (the merged-assembly schedule, whose tiles must lie in one
// row) a row of nx elements holds txn = ceil(nx/epb) tiles, the last one short,
// so tiles never straddle rows whatever nx is.
//
// Plain constexpr arithmetic, so host code (list building, tests) and device
// code evaluate the same function.
#pragma once

#include <cstdint>

namespace hb {

struct TileWalk {
    uint32_t txn = 0, ny = 0, nz = 0, ys = 0;  // txn == 0: identity (plain element order)
    uint32_t rowlen = 0;  // nonzero: padded rows of rowlen elements (txn tiles each, the last short)
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
// where a tile would straddle two rows: padded rows if pad, else identity.
constexpr TileWalk make_walk(int64_t nx, int64_t ny, int64_t nz, int epb, bool pad = false)
{
    TileWalk w;
    if (epb < 1 || nx < 0) return w;
    if (nx % epb != 0) {
        if (!pad) return w;
        w.rowlen = static_cast<uint32_t>(nx);
    }
    w.txn = static_cast<uint32_t>((nx + epb - 1) / epb);
    w.ny = static_cast<uint32_t>(ny);
    w.nz = static_cast<uint32_t>(nz);
    w.ys = static_cast<uint32_t>((ny + 7) / 8);  // one slab per XCD
    return w;
}

// Tiles of a launch over E elements.
constexpr int64_t walk_tiles(const TileWalk &w, int64_t E, int epb)
{
    return w.txn ? static_cast<int64_t>(w.txn) * w.ny * w.nz : (E + epb - 1) / epb;
}

// The elements of tile t (a value of walk_tile): e0 .. e0 + n - 1, n >= 1.
struct TileSpan {
    int64_t e0;
    int32_t n;
};
constexpr TileSpan tile_span(const TileWalk &w, uint32_t t, int64_t E, int epb)
{
    if (w.rowlen) {
        const uint32_t row = t / w.txn;
        const uint32_t k = (t - row * w.txn) * static_cast<uint32_t>(epb);  // offset in the row
        const uint32_t left = w.rowlen - k;
        return TileSpan{static_cast<int64_t>(row) * w.rowlen + k,
                        static_cast<int32_t>(left < static_cast<uint32_t>(epb) ? left : static_cast<uint32_t>(epb))};
    }
    const int64_t e0 = static_cast<int64_t>(t) * epb;
    const int64_t left = E - e0;
    return TileSpan{e0, static_cast<int32_t>(left < epb ? left : epb)};
}

}  // namespace hb
