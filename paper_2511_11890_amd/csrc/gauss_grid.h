// Launch geometry of the fused Gaussian (shared by the kernels and the host
// code that sizes the sigma-gradient partials).
#pragma once

#include "common.h"

namespace harpia {
namespace gauss_detail {

constexpr int kTX = 64;  // tile columns (x)
constexpr int kTY = 16;  // tile rows (y)

struct FusedGrid {
    int tiles_x, tiles_y, zlen;
    int64_t blocks;
};

inline FusedGrid fused_grid(const ChunkArgs &a, int R)
{
    FusedGrid g;
    g.tiles_x = (int)((a.out_e[2] + kTX - 1) / kTX);
    g.tiles_y = (int)((a.out_e[1] + kTY - 1) / kTY);
    const int64_t tiles = (int64_t)g.tiles_x * g.tiles_y;
    // z range per workgroup: enough workgroups to fill the chip several
    // times over, but long enough that the 2r-slice warm-up stays small.
    int64_t zlen = a.out_e[0];
    const int64_t want_blocks = 4096;
    if (tiles < want_blocks) {
        int64_t nzc = (want_blocks + tiles - 1) / tiles;
        zlen = (a.out_e[0] + nzc - 1) / nzc;
        const int64_t min_len = 8 * R > 32 ? 8 * R : 32;
        if (zlen < min_len) zlen = min_len;
    } else {
        const int64_t max_len = 256;
        if (zlen > max_len && tiles < 4 * want_blocks) zlen = max_len;
    }
    if (zlen > a.out_e[0]) zlen = a.out_e[0];
    g.zlen = (int)zlen;
    g.blocks = tiles * ((a.out_e[0] + zlen - 1) / zlen);
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
