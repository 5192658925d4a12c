// Tile footprints: the tile box of a splat and the trims of its rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sd7 {

// Tile footprint of a splat: its tile box and, for up to eight of the box's
// tile rows, how many tiles at the left and at the right end of the row the
// splat's opacity ellipse misses.  x = x0 | y0 << 16, y = x1 | y1 << 16 (x1,
// y1 exclusive); z holds rows 0..3, w rows m..m+3 with m = h - 4 for a box of
// h > 8 rows (else m = 4); byte = left | right << 4.  Rows 4..m-1 are whole.
struct Footprint {
    uint32_t x0, y0, x1, y1, top, bot;
    __device__ __forceinline__ explicit Footprint(uint4 f)
        : x0(f.x & 0xFFFFu), y0(f.x >> 16), x1(f.y & 0xFFFFu), y1(f.y >> 16), top(f.z), bot(f.w) {}
    __device__ __forceinline__ uint32_t h() const { return y1 - y0; }
    __device__ __forceinline__ uint32_t w() const { return x1 - x0; }
    __device__ __forceinline__ uint32_t first_bottom_row() const { return h() > 8 ? h() - 4 : 4; }
    // trim byte of row r (0 <= r < h); selects only, no lane branches
    __device__ __forceinline__ uint32_t trim(uint32_t r) const
    {
        const uint32_t m = first_bottom_row();
        const bool in_top = r < 4, in_bot = r >= m;
        const uint32_t word = in_top ? top : bot;
        const uint32_t byte = (word >> (8 * ((in_top ? r : r - m) & 3u))) & 0xFFu;
        return (in_top || in_bot) ? byte : 0u;
    }
    // tile columns [a, b) of row r; empty when a >= b
    __device__ __forceinline__ void row(uint32_t r, int& a, int& b) const
    {
        const uint32_t t = trim(r);
        a = (int)(x0 + (t & 15u));
        b = (int)x1 - (int)(t >> 4);
    }
    __device__ __forceinline__ uint32_t row_tiles(uint32_t r) const
    {
        int a, b;
        row(r, a, b);
        return b > a ? (uint32_t)(b - a) : 0u;
    }
    __device__ __forceinline__ bool trimmed() const { return (top | bot) != 0u; }
    // tiles of the footprint
    __device__ __forceinline__ uint32_t tiles() const
    {
        if (!trimmed()) return w() * h();
        const uint32_t hh = h(), m = first_bottom_row();
        uint32_t n = 0;
        for (uint32_t r = 0; r < 4 && r < hh; ++r) n += row_tiles(r);
        for (uint32_t r = m; r < hh; ++r) n += row_tiles(r);
        return n + (m > 4 ? (m - 4) * w() : 0u);
    }
};

}  // namespace sd7
