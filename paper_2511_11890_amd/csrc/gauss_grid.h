// Launch geometry of the fused Gaussian (shared by the kernels and the host
// code that sizes the sigma-gradient partials).
#pragma once

#include <algorithm>

#include "common.h"

namespace harpia {
namespace gauss_detail {

constexpr int kTX = 64;  // tile columns (x)
constexpr int kTY = 16;  // tile rows (y)

// Tile width of the plain fused Gaussian: 128 columns (512 threads) for
// radii up to 6, so a patch row spans fewer partial 128-byte lines per
// output; 64 columns (256 threads) above, where the register ring and the
// LDS patch grow with r.
constexpr int fused_tx(int r) { return r <= 6 ? 128 : 64; }

struct FusedGrid {
    int tiles_x, tiles_y, zlen;
    int64_t blocks;
};

// Largest number of z ranges a launch uses (bounds the sigma-gradient
// partials: one per workgroup).
constexpr int64_t kMaxZRanges = 64;

// ranges > 0: split z into that many ranges (the autotuner's choice).
inline FusedGrid fused_grid(const ChunkArgs &a, int R, int64_t capacity, int ranges = 0, int tx = kTX)
{
    FusedGrid g;
    g.tiles_x = (int)((a.out_e[2] + tx - 1) / tx);
    g.tiles_y = (int)((a.out_e[1] + kTY - 1) / kTY);
    const int64_t tiles = (int64_t)g.tiles_x * g.tiles_y;
    int64_t nzc = z_ranges(a.out_e[0], tiles, capacity, R, kMaxZRanges);
    if (ranges > 0) nzc = std::min<int64_t>(std::min<int64_t>(ranges, a.out_e[0]), kMaxZRanges);
    g.zlen = (int)((a.out_e[0] + nzc - 1) / nzc);
    g.blocks = tiles * ((a.out_e[0] + g.zlen - 1) / g.zlen);
    return g;
}

inline bool fused_ok(const GaussTaps &t, const ChunkArgs &a)
{
    if (!(t.r[0] == t.r[1] && t.r[1] == t.r[2])) return false;
    if (t.r[0] < 1 || t.r[0] > kGaussFusedMaxR) return false;
    // in-plane offsets are 32-bit
    return a.in_sy * (a.n[1] + 1) < (int64_t)1 << 31;
}

}  // namespace gauss_detail
}  // namespace harpia
