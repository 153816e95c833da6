// Launch geometry of the fused Gaussian (shared by the kernels and the host
// code that sizes the sigma-gradient partials).
#pragma once

#include <algorithm>

#include "common.h"

namespace harpia {
namespace gauss_detail {

constexpr int kTX = 64;  // tile columns (x)
constexpr int kTY = 16;  // tile rows (y)

// Tile width of the plain fused Gaussian: 256 columns (1024 threads) for
// radii up to 4, 128 columns (512 threads) above.  Wider tiles stage fewer
// x-halo columns per output (the y pass filters TX + 2r columns) and span
// fewer partial 128-byte lines per patch row; at radius 5 and up a
// 1024-thread workgroup's 128-register cap would spill the z ring (at
// radius 4 already with the unsharp epilogue's extra registers).
constexpr int fused_tx(int r, bool unsharp = false) { return r <= (unsharp ? 3 : 4) ? 256 : 128; }

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

// In-plane offsets of the fused kernels are 32-bit.
inline bool fused_ok_extent(const ChunkArgs &a) { return a.in_sy * (a.n[1] + 1) < (int64_t)1 << 31; }

inline bool fused_ok(const GaussTaps &t, const ChunkArgs &a)
{
    if (!(t.r[0] == t.r[1] && t.r[1] == t.r[2])) return false;
    if (t.r[0] < 1 || t.r[0] > kGaussFusedMaxR) return false;
    return fused_ok_extent(a);
}

}  // namespace gauss_detail
}  // namespace harpia
