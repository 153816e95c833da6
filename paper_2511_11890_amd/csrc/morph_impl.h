// Erosion / dilation kernels for gfx950 (the label-editing module's
// morphology, Section III-C).  Templates; instantiated per input dtype in
// morph_<dtype>.hip so the build compiles them in parallel.
//
// Definitions: dilation takes the max, erosion the min, of the input over the
// structuring element B placed at the voxel; B is a box |d_a| <= r or a ball
// dz^2 + dy^2 + dx^2 <= r^2.  At the faces the input is reflected
// (half-sample), which for these elements gives the same result as ignoring
// offsets outside the volume.
//
// Single-op kernels compute a dilation; an erosion is the dilation of the
// negated input, negated back (exact for every dtype: negation is exact in
// f32 and all u8/u16/f16/bf16 values are f32 values; the fast grayscale
// kernels complement the order keys instead, which is the same reversal).
// Binary erosion is the complement of the dilation of the complement.
// "Both" kernels return the erosion and the dilation from one read of the
// input.  Grayscale extrema follow the IEEE 754 totalOrder of the values
// (order_key).
//
// Structure (same skeleton as the fused Gaussian): a 256-thread workgroup
// owns a tile of output columns and streams along z.  Per input slice:
//   1. the (tile + 2r halo) patch is staged in LDS (reflection on load);
//   2. stage A: x-run extrema of half-width h for every level h the element
//      needs (box: h = r only; ball: h = 0..r), from LDS, into LDS planes;
//   3. stage B: for every z-class c = |dz| the in-plane disc (ball: rows
//      |dy| <= floor(sqrt(r^2 - c^2)) with x half-width
//      floor(sqrt(r^2 - c^2 - dy^2)); box: the full square) is the extremum
//      of the level planes over its rows;
//   4. z: a register ring of 2r+1 running extrema per column; slice s feeds
//      class |o - s| into output o, and output s - r is complete.
// Binary data runs on bit rows (bits_kernel): a lane holds a row of 64
// voxels as a 64-bit mask, extrema become OR on masks, x shifts are mask
// shifts and y neighbours come from other lanes by cross-lane shuffles.
#pragma once

#include <cstdint>
#include <utility>

#include "common.h"
#include "batch.h"
#include "tune.h"

namespace harpia {


namespace morph_detail {

constexpr int kNT = 256;
constexpr int kMaxFastR = 4;

constexpr int isqrt_c(int v)
{
    int r = 0;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// Geometry of the element: z-classes, their y half-extent and the x
// half-width of each of their rows.
template <int SE, int R>
struct Shape {
    static constexpr int NC = (SE == HARPIA_SE_BOX) ? 1 : R + 1;  // z-classes
    static constexpr int NL = (SE == HARPIA_SE_BOX) ? 1 : R + 1;  // x-run levels
    static constexpr int cls(int d) { return SE == HARPIA_SE_BOX ? 0 : (d < 0 ? -d : d); }
    static constexpr int rho(int c) { return SE == HARPIA_SE_BOX ? R : isqrt_c(R * R - c * c); }
    static constexpr int hw(int c, int dy)
    {
        return SE == HARPIA_SE_BOX ? R : isqrt_c(R * R - c * c - dy * dy);
    }
    static constexpr int lvl(int h) { return SE == HARPIA_SE_BOX ? 0 : h; }
    // Widest x-run any class needs on row dy (-1: none), and whether some
    // class takes the run of half-width h on row dy.
    static constexpr int max_hw(int dy)
    {
        int m = -1;
        for (int c = 0; c < NC; ++c)
            if ((dy < 0 ? -dy : dy) <= rho(c) && hw(c, dy) > m) m = hw(c, dy);
        return m;
    }
    static constexpr bool takes(int c, int dy, int h) { return (dy < 0 ? -dy : dy) <= rho(c) && hw(c, dy) == h; }
};

// Grid shape shared by the launchers: tiles of TX x TY columns, z ranges
// long enough to amortise the 2r-slice warm-up, enough workgroups to fill
// the chip.
struct Grid {
    int tiles_x, tiles_y;
    int zlen;
    int64_t blocks;
};

// ranges > 0: split z into that many ranges (the autotuner's choice).
inline Grid make_grid(const ChunkArgs &a, int TX, int TY, int R, int64_t capacity, int ranges = 0)
{
    Grid g;
    g.tiles_x = (int)((a.out_e[2] + TX - 1) / TX);
    g.tiles_y = (int)((a.out_e[1] + TY - 1) / TY);
    const int64_t tiles = (int64_t)g.tiles_x * g.tiles_y;
    int64_t nzc = z_ranges(a.out_e[0], tiles, capacity, R);
    if (ranges > 0) nzc = ranges < a.out_e[0] ? ranges : a.out_e[0];
    g.zlen = (int)((a.out_e[0] + nzc - 1) / nzc);
    g.blocks = tiles * ((a.out_e[0] + g.zlen - 1) / g.zlen);
    return g;
}

// ------------------------------------------------------------- grayscale

constexpr int kGTX = 64, kGTY = 16;
constexpr int kGC = 2;                            // output columns per thread
constexpr int kGNT = (kGTX / kGC) * kGTY;         // threads per workgroup

// Order-preserving map of a float to a signed int: the bit pattern with the
// 31 value bits inverted when the sign bit is set, so that int order is the
// IEEE 754 totalOrder of the values (-0 < +0, NaNs beyond the infinities by
// their sign).  The map is its own inverse.  Grayscale extrema are taken on
// these keys: integer min / max are exact like the float ones and, unlike
// them, need no quieting of signalling NaNs before every operation.
__device__ __forceinline__ int order_key(float x)
{
    const int b = __float_as_int(x);
    return b ^ (int)((uint32_t)(b >> 31) >> 1);
}
__device__ __forceinline__ float order_value(int k) { return __int_as_float(k ^ (int)((uint32_t)(k >> 31) >> 1)); }

// Second output of the "both" kernels.
struct Out2 {
    void *ptr;
    int64_t sy, sz;
};

template <typename T, int SE, int R, bool BOTH, int TX = kGTX>
__device__ __forceinline__ void gray_tile(const ChunkArgs &a, const Out2 &o2, float sign, int zlen, int bx, int by,
                                          int bz)
{
    using S = Shape<SE, R>;
    constexpr int NT = TX / kGC * kGTY;  // threads: kGC columns each
    constexpr int P = 2 * R + 1;
    constexpr int PW = TX + 2 * R;
    constexpr int PWP = (PW + 3) & ~3;
    constexpr int PH = kGTY + 2 * R;
    constexpr int PSZ = PW * PH;
    constexpr int NLD = (PSZ + NT - 1) / NT;
    constexpr int NV = kGC + 2 * R;               // patch columns one thread reads per row
    constexpr int NV4 = (NV + 3) / 4;
    constexpr int NM = BOTH ? 2 : 1;      // 0: max (dilation), 1: min
    constexpr int BUF = PH * PWP + 4 * NV4;

    // Double-buffered patch of order keys: slice i is staged into sP[i & 1]
    // while other threads may still read slice i - 1 from the other half, so
    // one barrier per slice suffices.  Every thread derives the x-runs it
    // needs straight from the patch (no intermediate LDS arrays).  A
    // single-op erosion stages the complemented keys (which reverse the
    // order) and takes maxima.
    __shared__ __attribute__((aligned(16))) int sP[2 * BUF];
    const int flip = (!BOTH && sign < 0.f) ? -1 : 0;

    const int tid = threadIdx.x;
    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * TX;
    const int64_t y0 = ybeg + (int64_t)by * kGTY;
    const int64_t zo0 = a.out_o[0] + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, a.out_o[0] + a.out_e[0]);
    if (zo0 >= zo1) return;

    int32_t off[NLD];
    int32_t lds[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * NT;
        off[i] = 0;
        lds[i] = 0;
        if (e < PSZ) {
            const int row = e / PW, col = e - (e / PW) * PW;
            int64_t gy = y0 - R + row;
            gy = gy < ybeg - R ? ybeg - R : (gy > yend - 1 + R ? yend - 1 + R : gy);
            int64_t gx = x0 - R + col;
            gx = gx < xbeg - R ? xbeg - R : (gx > xend - 1 + R ? xend - 1 + R : gx);
            off[i] = (int32_t)((reflect_index(gy, a.n[1]) - a.in_o[1]) * a.in_sy +
                               (reflect_index(gx, a.n[2]) - a.in_o[2]));
            lds[i] = row * PWP + col;
        }
    }

    const int64_t s0 = zo0 - R;
    const int nsteps = (int)(zo1 - zo0) + 2 * R;
    const T *in = static_cast<const T *>(a.in);
    // The next slice's raw values (converted when staged, so the loads stay
    // in flight through a whole step).  The fetch is unconditional: past the
    // last slice it re-reads that slice, which is never used.
    T pf[NLD];
    auto fetch = [&](int j) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const T *base = in + (reflect_index(s0 + j, a.n[0]) - a.in_o[0]) * a.in_sz;
#pragma unroll
        for (int i = 0; i < NLD; ++i)
            if (i < NLD - 1 || tid + i * NT < PSZ) pf[i] = base[off[i]];
    };

    const int qrow = tid / (TX / kGC);
    const int qcol = (tid % (TX / kGC)) * kGC;
    const int64_t gy_out = y0 + qrow;
    const int64_t gx_out = x0 + qcol;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)kGC, xend - gx_out) : 0;
    T *outp = static_cast<T *>(a.out) + (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);
    T *outp2 = BOTH ? static_cast<T *>(o2.ptr) + (gy_out - ybeg) * o2.sy + (gx_out - xbeg) : nullptr;

    int acc[NM][P][kGC];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < kGC; ++c) acc[m][j][c] = 0;

    fetch(0);

    // Step i (0 .. nsteps): stage slice i and fetch slice i + 1, store the
    // output completed by step i - 1 (after the fetch, so that the next
    // staging waits only for work issued a step earlier), then filter slice i.
    for (int base = 0; base <= nsteps; base += P) {
        static_for<P>([&](auto U) {
            constexpr int u = decltype(U)::value;
            const int i = base + u;
            if (i > nsteps) return;
            int *buf = sP + (i & 1) * BUF;
            if (i < nsteps) {
#pragma unroll
                for (int k = 0; k < NLD; ++k)
                    if (k < NLD - 1 || tid + k * NT < PSZ) buf[lds[k]] = order_key(to_f32(pf[k])) ^ flip;
                fetch(i + 1);
            }
            if (i >= 1 && i - 1 >= 2 * R && nvalid > 0) {
                constexpr int sl = (u - 1 - R + 2 * P) % P;
                const int64_t zl = s0 + (i - 1) - R - a.out_o[0];
                if constexpr (BOTH) {
                    // out = erosion (min), out2 = dilation (max)
#pragma unroll
                    for (int q = 0; q < kGC; ++q)
                        if (q < nvalid) {
                            outp[zl * a.out_sz + q] = from_f32<T>(order_value(acc[1][sl][q]));
                            outp2[zl * o2.sz + q] = from_f32<T>(order_value(acc[0][sl][q]));
                        }
                } else {
#pragma unroll
                    for (int q = 0; q < kGC; ++q)
                        if (q < nvalid) outp[zl * a.out_sz + q] = from_f32<T>(order_value(acc[0][sl][q] ^ flip));
                }
            }
            if (i >= nsteps) return;
            lds_barrier();

            // In-plane disc of every z-class (kGC columns): rows dy = -R .. R,
            // each row's x-runs of the half-widths its classes take.
            int disc[NM][S::NC][kGC];
            static_for<P>([&](auto DY) {
                constexpr int dy = decltype(DY)::value - R;
                constexpr int hmax = S::max_hw(dy);
                if constexpr (hmax >= 0) {
                    int v[NV4 * 4];
                    const int *prow = &buf[(qrow + R + dy) * PWP + qcol];
                    if constexpr (kGC % 4 == 0) {
                        const int4 *p4 = reinterpret_cast<const int4 *>(prow);
#pragma unroll
                        for (int j = 0; j < NV4; ++j) {
                            const int4 t4 = p4[j];
                            v[4 * j] = t4.x;
                            v[4 * j + 1] = t4.y;
                            v[4 * j + 2] = t4.z;
                            v[4 * j + 3] = t4.w;
                        }
                    } else {
                        const int2 *p2 = reinterpret_cast<const int2 *>(prow);
#pragma unroll
                        for (int j = 0; j < 2 * NV4; ++j) {
                            const int2 t2 = p2[j];
                            v[2 * j] = t2.x;
                            v[2 * j + 1] = t2.y;
                        }
                    }
#pragma unroll
                    for (int m = 0; m < NM; ++m) {
                        int run[kGC];
#pragma unroll
                        for (int q = 0; q < kGC; ++q) run[q] = v[q + R];
                        static_for<hmax + 1>([&](auto H) {
                            constexpr int h = decltype(H)::value;
                            if constexpr (h > 0) {
#pragma unroll
                                for (int q = 0; q < kGC; ++q)
                                    run[q] = (m == 0) ? max(run[q], max(v[q + R - h], v[q + R + h]))
                                                      : min(run[q], min(v[q + R - h], v[q + R + h]));
                            }
                            static_for<S::NC>([&](auto C) {
                                constexpr int c = decltype(C)::value;
                                if constexpr (S::takes(c, dy, h)) {
                                    constexpr bool first = (dy == -S::rho(c));
#pragma unroll
                                    for (int q = 0; q < kGC; ++q)
                                        disc[m][c][q] = first ? run[q]
                                                              : ((m == 0) ? max(disc[m][c][q], run[q])
                                                                          : min(disc[m][c][q], run[q]));
                                }
                            });
                        });
                    }
                }
            });
            // z ring: slice i feeds the outputs i + d (offset -d) of each class;
            // every slot takes one contribution per slice, slot (u + R) its first
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                static_for<P>([&](auto DD) {
                    constexpr int d = decltype(DD)::value - R;
                    constexpr int c = S::cls(d);
                    constexpr int sl = (u + d + 2 * P) % P;
#pragma unroll
                    for (int q = 0; q < kGC; ++q)
                        acc[m][sl][q] = (d == R) ? disc[m][c][q]
                                                 : ((m == 0) ? max(acc[m][sl][q], disc[m][c][q])
                                                             : min(acc[m][sl][q], disc[m][c][q]));
                });
            }
        });
    }
}

// Tile width of the single-volume kernel: 128 columns (1024 threads) up to
// radius 3, so a patch row spans fewer partial 128-byte lines per output;
// 64 columns (512 threads) at radius 4, whose registers would not fit the
// wider workgroup.
constexpr int gray_tx(int r) { return r <= 3 ? 128 : kGTX; }
constexpr int gray_nt(int r) { return gray_tx(r) / kGC * kGTY; }

template <typename T, int SE, int R, bool BOTH>
__global__ __launch_bounds__(gray_nt(R)) void gray_kernel(ChunkArgs a, Out2 o2, float sign, int tiles_x, int tiles_y,
                                                   int zlen)
{
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(b % (uint32_t)tiles_x);
    const int by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(b / (uint32_t)(tiles_x * tiles_y));
    gray_tile<T, SE, R, BOTH, gray_tx(R)>(a, o2, sign, zlen, bx, by, bz);
}

// Persistent batched grayscale morphology (in -> out, aux -> second output
// of a "both" step; the same element for every crop).
template <typename T, int SE, int R, bool BOTH>
__global__ __launch_bounds__(kGNT) void gray_batched_kernel(BatchDesc d, float sign)
{
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const ChunkArgs a = crop_args(d.c[c]);
        const Out2 o2{const_cast<void *>(d.c[c].aux), a.out_sy, a.out_sz};
        gray_tile<T, SE, R, BOTH>(a, o2, sign, d.c[c].zlen, bx, by, bz);
        lds_barrier();
    }
}

// ---------------------------------------------------------------- binary

// Binary erosion / dilation on bit rows.
//
// A wave owns a strip of kBX = 64 output columns and streams along z; lane l
// holds input row y_w - R + l of the strip (64 rows: the wave's 64 - 2R
// output rows plus R halo rows on each side).  The four waves of a workgroup
// take four neighbouring strips of the same rows, so that the bytes of a
// row they read and write (a whole 256-voxel span) share cache lines at the
// same time.  A row
// of a slice is one 64-bit mask (bit i: voxel x0 + i is set) plus the 4
// voxels on each side (enough for R <= 4).  Dilation:
//   x runs      D_h = OR over |k| <= h of the row shifted by k (mask shifts
//               with the halo bits carried in);
//   discs       for each z-class c = |dz|, the OR over rows |dy| <= rho_c of
//               D_{hw(c, dy)} of row y + dy, taken from lane l + dy by a
//               cross-lane shuffle;
//   z           a ring of 2R + 1 running ORs per lane; slice s feeds the
//               disc of class |o - s| into output o, and output s - R is then
//               complete and written as bytes.
// Erosion is the complement of the dilation of the complement.  Voxels
// outside the volume are 0 in the mask that is dilated (for these elements
// ignoring them is the reflect boundary), and so are voxels farther than R
// from the output region (no stored output reads them).  No barriers:
// the waves are independent (each has a private LDS block through which its
// output rows reach coalesced stores).
// 1 if v counts as set: v > thr (use_thr; thr is the largest value of the
// input's type not above the threshold, so the comparison is exact) or v != 0.
template <typename Tin>
__device__ __forceinline__ uint32_t binarise(Tin v, float thr, bool use_thr)
{
    const float f = to_f32(v);
    return use_thr ? (f > thr ? 1u : 0u) : (f != 0.f ? 1u : 0u);
}

constexpr int kBX = 64;               // output columns per wave
constexpr int kBG = kBX / 4 + 2;      // 4-voxel groups per row: halo, 16 core, halo
constexpr int kBNT = 256;             // threads per workgroup (4 waves)

template <int R>
constexpr int bits_rows() { return 64 - 2 * R; }  // output rows per wave

// Raw storage of one 4-voxel group: 4 elements of Tin.
template <typename Tin>
struct Group4 {
    static constexpr int W = (int)sizeof(Tin);  // 32-bit words per group
    uint32_t w[W];
};

template <typename Tin>
__device__ __forceinline__ Tin group_elem(const Group4<Tin> &g, int j)
{
    Tin v;
    __builtin_memcpy(&v, reinterpret_cast<const char *>(g.w) + j * sizeof(Tin), sizeof(Tin));
    return v;
}

template <typename Tin>
__device__ __forceinline__ void group_load4(Group4<Tin> &g, const Tin *p)
{
    if constexpr (sizeof(Tin) == 1) {
        g.w[0] = *reinterpret_cast<const uint32_t *>(p);
    } else if constexpr (sizeof(Tin) == 2) {
        const uint2 t = *reinterpret_cast<const uint2 *>(p);
        g.w[0] = t.x;
        g.w[1] = t.y;
    } else {
        const uint4 t = *reinterpret_cast<const uint4 *>(p);
        g.w[0] = t.x;
        g.w[1] = t.y;
        g.w[2] = t.z;
        g.w[3] = t.w;
    }
}

// Elements j, j + 1 of a group from one load (2-element alignment).
template <typename Tin>
__device__ __forceinline__ void group_load2(Group4<Tin> &g, int j, const Tin *p)
{
    if constexpr (sizeof(Tin) == 1) {
        const uint16_t t = *reinterpret_cast<const uint16_t *>(p);
        __builtin_memcpy(reinterpret_cast<char *>(g.w) + j, &t, 2);
    } else if constexpr (sizeof(Tin) == 2) {
        g.w[j >> 1] = *reinterpret_cast<const uint32_t *>(p);
    } else {
        const uint2 t = *reinterpret_cast<const uint2 *>(p);
        g.w[j] = t.x;
        g.w[j + 1] = t.y;
    }
}

template <typename Tin>
__device__ __forceinline__ void group_set(Group4<Tin> &g, int j, Tin v)
{
    __builtin_memcpy(reinterpret_cast<char *>(g.w) + j * sizeof(Tin), &v, sizeof(Tin));
}

// Bits of a group of 4 voxels (bit k: voxel k) that lies wholly inside the
// read window: v > thr_i for integer inputs (thr_i the threshold's floor, so
// the comparison is exact), v > thr for float inputs, or v != 0.
template <typename Tin>
__device__ __forceinline__ uint32_t group_bits(const Group4<Tin> &g, float thr, int thr_i, bool use_thr)
{
    uint32_t nib = 0;
    if constexpr (std::is_same<Tin, uint8_t>::value) {
        const uint32_t w = g.w[0];
        if (!use_thr) {
            // bit 7 of each byte: byte != 0; then gather bits 7, 15, 23, 31
            const uint32_t t = ((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w;
            return (((t >> 7) & 0x01010101u) * 0x01020408u) >> 24;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) nib |= (((int)((w >> (8 * k)) & 0xffu) > thr_i) ? 1u : 0u) << k;
    } else if constexpr (std::is_same<Tin, uint16_t>::value) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int v = (int)((g.w[k >> 1] >> (16 * (k & 1))) & 0xffffu);
            nib |= ((use_thr ? v > thr_i : v != 0) ? 1u : 0u) << k;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) nib |= binarise(group_elem<Tin>(g, k), thr, use_thr) << k;
    }
    return nib;
}

// 16 output bytes (voxel order) from 16 bits.
__device__ __forceinline__ uint4 bits_to_bytes16(uint32_t b)
{
    // nibble n (bits b3 b2 b1 b0) -> bytes b0 b1 b2 b3: the four shifted
    // copies of n * 0x204081 do not overlap, so bit 8j holds b_j
    uint32_t q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = (((b >> (4 * j)) & 0xfu) * 0x204081u) & 0x01010101u;
    return make_uint4(q[0], q[1], q[2], q[3]);
}

// 16-byte store marked non-temporal: output rows are not read back by the
// kernel, so they need not displace the input rows from the caches.
__device__ __forceinline__ void store16_nt(uint8_t *p, uint4 v)
{
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<v4u *>(p));
}

template <typename Tin, int SE, int R, bool BOTH>
__global__ __launch_bounds__(kBNT) void bits_kernel(ChunkArgs a, Out2 o2, uint32_t flip, float thr, int use_thr,
                                                    int vec_in, int vec_out, int tiles_x, int tiles_y, int zlen)
{
    static_assert(R >= 1 && R <= 4, "4 halo voxels per side");
    using S = Shape<SE, R>;
    constexpr int P = 2 * R + 1;
    constexpr int NM = BOTH ? 2 : 1;  // pipeline m = 0: dilation of b (BOTH) or of b ^ flip; m = 1: of ~b
    constexpr int YR = bits_rows<R>();

    // the wave index is uniform across a wave: keep it (and the strip's
    // window tests) in scalar registers
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(b % (uint32_t)tiles_x);
    const int by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(b / (uint32_t)(tiles_x * tiles_y));

    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1], zbeg = a.out_o[0];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1], zend = zbeg + a.out_e[0];
    const int64_t x0 = xbeg + ((int64_t)bx * 4 + wave) * kBX;
    const int64_t yw = ybeg + (int64_t)by * YR;  // first output row of this wave
    const int64_t zo0 = zbeg + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, zend);
    if (zo0 >= zo1 || x0 >= xend) return;

    // window of voxels that may be read: the volume, within R of the output
    // region
    const int64_t xlo = max((int64_t)0, xbeg - R), xhi = min(a.n[2], xend + R);
    const int64_t ylo = max((int64_t)0, ybeg - R), yhi = min(a.n[1], yend + R);
    const int64_t zlo = max((int64_t)0, zbeg - R), zhi = min(a.n[0], zend + R);

    const int64_t y = yw - R + lane;
    const bool row_in = y >= ylo && y < yhi;
    const Tin *in = static_cast<const Tin *>(a.in);
    const Tin *row_base = in + (row_in ? (y - a.in_o[1]) * a.in_sy : 0) - a.in_o[2];

    // in-window mask of the strip (the same for every lane): bit k of the
    // group-g nibble is voxel x0 - 4 + 4 g + k
    auto in_x = [&](int64_t x) __attribute__((always_inline)) { return x >= xlo && x < xhi; };

    const int64_t s0 = zo0 - R;
    const int nsteps = (int)(zo1 - zo0) + 2 * R;
    const int thr_i = (int)thr;  // integer inputs: thr is the threshold's floor

    // The wave's LDS block passes each output row from its lane to
    // coalesced stores: 16 rows of 64 bytes per store instruction instead of
    // 64 rows of 16 (row pitch of 20 words: b128 writes on distinct banks).
    constexpr int kOutPitch = 20;
    __shared__ __attribute__((aligned(16))) uint32_t sB[4][64 * kOutPitch];
    uint32_t *blk = sB[wave];
    Group4<Tin> raw[kBG];
    auto load_group = [&](const Tin *p, int g) __attribute__((always_inline)) {
        const int64_t xg = x0 - 4 + 4 * g;
        if (vec_in >= 4 && in_x(xg) && in_x(xg + 3)) {
            group_load4<Tin>(raw[g], p + xg);
        } else if (vec_in == 2 && in_x(xg) && in_x(xg + 3)) {
            group_load2<Tin>(raw[g], 0, p + xg);
            group_load2<Tin>(raw[g], 2, p + xg + 2);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (in_x(xg + k)) group_set<Tin>(raw[g], k, p[xg + k]);
        }
    };
    auto fetch = [&](int j) __attribute__((always_inline)) {
        const int64_t z = s0 + (j < nsteps ? j : nsteps - 1);
        if (!row_in || z < zlo || z >= zhi) return;
        const Tin *p = row_base + (z - a.in_o[0]) * a.in_sz;
        if constexpr (sizeof(Tin) <= 2) {
            // 16-byte aligned rows with the whole 64-voxel core in the
            // window: the core in 16-byte loads (4 for u8, 8 for 16-bit
            // types) instead of one load per 4-voxel group
            if (vec_in == 16 && in_x(x0) && in_x(x0 + kBX - 1)) {
                constexpr int GW = Group4<Tin>::W;
                const uint4 *q = reinterpret_cast<const uint4 *>(p + x0);
#pragma unroll
                for (int i = 0; i < kBX * (int)sizeof(Tin) / 16; ++i) {
                    const uint4 t = q[i];
                    const uint32_t w4[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) raw[1 + (4 * i + k) / GW].w[(4 * i + k) % GW] = w4[k];
                }
                load_group(p, 0);
                load_group(p, kBG - 1);
                return;
            }
        }
#pragma unroll
        for (int g = 0; g < kBG; ++g) load_group(p, g);
    };
    // bits of slice j from raw: row mask, left halo (bits 0..3 = x0-4..x0-1),
    // right halo (bits 0..3 = x0+64..x0+67); 0 outside the window.  Returns
    // whether the row lies in the window (else its complement is 0 too).
    auto pack = [&](int j, uint64_t &m, uint32_t &hl, uint32_t &hr) __attribute__((always_inline)) -> bool {
        m = 0;
        hl = hr = 0;
        const int64_t z = s0 + j;
        if (!row_in || z < zlo || z >= zhi) return false;
#pragma unroll
        for (int g = 0; g < kBG; ++g) {
            const int64_t xg = x0 - 4 + 4 * g;
            uint32_t nib = 0;
            if (in_x(xg) && in_x(xg + 3)) {
                nib = group_bits<Tin>(raw[g], thr, thr_i, use_thr);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (in_x(xg + k)) nib |= binarise(group_elem<Tin>(raw[g], k), thr, use_thr) << k;
            }
            if (g == 0)
                hl = nib;
            else if (g == kBG - 1)
                hr = nib;
            else
                m |= (uint64_t)nib << (4 * (g - 1));
        }
        return true;
    };
    // window masks of the strip (for complements)
    uint64_t wm = 0;
    uint32_t wl = 0, wr = 0;
#pragma unroll
    for (int g = 0; g < kBG; ++g) {
        const int64_t xg = x0 - 4 + 4 * g;
        uint32_t nib = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (in_x(xg + k)) nib |= 1u << k;
        if (g == 0)
            wl = nib;
        else if (g == kBG - 1)
            wr = nib;
        else
            wm |= (uint64_t)nib << (4 * (g - 1));
    }

    const bool out_row = lane >= R && lane < 64 - R && y < yend;
    const int64_t nx_out = xend - x0;  // valid output columns of the strip (may exceed 64)
    uint8_t *outp = static_cast<uint8_t *>(a.out) + (y - ybeg) * a.out_sy + (x0 - xbeg);
    uint8_t *outp2 = BOTH ? static_cast<uint8_t *>(o2.ptr) + (y - ybeg) * o2.sy + (x0 - xbeg) : nullptr;
    auto emit = [&](uint8_t *p, uint64_t v) __attribute__((always_inline)) {
        if (vec_out == 16 && nx_out >= kBX) {
#pragma unroll
            for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(p)[q] = bits_to_bytes16((uint32_t)(v >> (16 * q)));
        } else if (vec_out == 4 && nx_out >= kBX) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 b4 = bits_to_bytes16((uint32_t)(v >> (16 * q)));
                uint32_t *p4 = reinterpret_cast<uint32_t *>(p) + 4 * q;
                p4[0] = b4.x;
                p4[1] = b4.y;
                p4[2] = b4.z;
                p4[3] = b4.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kBX; ++i)
                if (i < nx_out) p[i] = (uint8_t)((v >> i) & 1u);
        }
    };

    // Coalesced output of slice zl (whole 64-column strips with 16-byte
    // aligned rows): every lane puts its row's 64 bytes into the block, then
    // store k of lane l writes 16 bytes of row (64 k + l) / 4.  Rows that are
    // halo or past the region are not stored.
    auto emit_rows = [&](uint8_t *slice, int64_t sy, uint64_t v) __attribute__((always_inline)) {
        uint4 *mine = reinterpret_cast<uint4 *>(blk + lane * kOutPitch);
#pragma unroll
        for (int q = 0; q < 4; ++q) mine[q] = bits_to_bytes16((uint32_t)(v >> (16 * q)));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int idx = 64 * k + lane, r = idx >> 2, q = idx & 3;
            const int64_t yr = yw - R + r;
            const uint4 b4 = *reinterpret_cast<const uint4 *>(blk + r * kOutPitch + 4 * q);
            if (r >= R && r < 64 - R && yr < yend)
                store16_nt(slice + (yr - ybeg) * sy + 16 * q, b4);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const bool rows_out = vec_out == 16 && nx_out >= kBX;  // uniform per wave

    uint64_t acc[NM][P];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int j = 0; j < P; ++j) acc[m][j] = 0;

    fetch(0);
    for (int base = 0; base < nsteps; base += P) {
        static_for<P>([&](auto U) {
            constexpr int u = decltype(U)::value;
            const int i = base + u;
            if (i >= nsteps) return;
            uint64_t row[NM];
            uint32_t hl[NM], hr[NM];
            const bool live = pack(i, row[0], hl[0], hr[0]);
            fetch(i + 1);
            // complement within the window (voxels outside stay 0)
            const uint64_t cm = live ? wm : 0;
            const uint32_t cl = live ? wl : 0, cr = live ? wr : 0;
            if constexpr (BOTH) {
                row[1] = ~row[0] & cm;
                hl[1] = ~hl[0] & cl;
                hr[1] = ~hr[0] & cr;
            } else if (flip) {
                row[0] = ~row[0] & cm;
                hl[0] = ~hl[0] & cl;
                hr[0] = ~hr[0] & cr;
            }
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                // x runs of every half-width up to R
                uint64_t dlev[R + 1];
                dlev[0] = row[m];
#pragma unroll
                for (int h = 1; h <= R; ++h) {
                    const uint64_t up = (row[m] >> h) | ((uint64_t)hr[m] << (64 - h));    // voxel x + h
                    const uint64_t dn = (row[m] << h) | (uint64_t)(hl[m] >> (4 - h));     // voxel x - h
                    dlev[h] = dlev[h - 1] | up | dn;
                }
                // discs of the z-classes from the rows of lanes l + dy
                uint64_t disc[S::NC];
#pragma unroll
                for (int c = 0; c < S::NC; ++c) disc[c] = 0;
                static_for<P>([&](auto DY) {
                    constexpr int dy = decltype(DY)::value - R;
                    static_for<R + 1>([&](auto H) {
                        constexpr int h = decltype(H)::value;
                        constexpr bool used = [] {
                            for (int c = 0; c < S::NC; ++c)
                                if (S::takes(c, dy, h)) return true;
                            return false;
                        }();
                        if constexpr (used) {
                            const uint64_t v = dy == 0 ? dlev[h] : (uint64_t)__shfl(dlev[h], lane + dy, 64);
                            static_for<S::NC>([&](auto C) {
                                constexpr int c = decltype(C)::value;
                                if constexpr (S::takes(c, dy, h)) disc[c] |= v;
                            });
                        }
                    });
                });
                // z ring: slice i feeds output s0 + i + d, slot (i + d) mod P
                static_for<P>([&](auto DD) {
                    constexpr int d = decltype(DD)::value - R;
                    constexpr int sl = (u + d + 2 * P) % P;
                    acc[m][sl] = (d == R) ? disc[S::cls(d)] : (acc[m][sl] | disc[S::cls(d)]);
                });
            }
            // output s0 + i - R is complete
            if (i >= 2 * R) {
                constexpr int sl = (u - R + 2 * P) % P;
                const int64_t o = s0 + i - R;
                if (o < zo1) {
                    const int64_t zl = o - zbeg;
                    if (rows_out) {
                        uint8_t *s1 = static_cast<uint8_t *>(a.out) + zl * a.out_sz + (x0 - xbeg);
                        if constexpr (BOTH) {
                            uint8_t *s2 = static_cast<uint8_t *>(o2.ptr) + zl * o2.sz + (x0 - xbeg);
                            emit_rows(s1, a.out_sy, ~acc[1][sl]);  // erosion
                            emit_rows(s2, o2.sy, acc[0][sl]);      // dilation
                        } else {
                            emit_rows(s1, a.out_sy, flip ? ~acc[0][sl] : acc[0][sl]);
                        }
                    } else if (out_row) {
                        if constexpr (BOTH) {
                            emit(outp + zl * a.out_sz, ~acc[1][sl]);  // erosion
                            emit(outp2 + zl * o2.sz, acc[0][sl]);     // dilation
                        } else {
                            emit(outp + zl * a.out_sz, flip ? ~acc[0][sl] : acc[0][sl]);
                        }
                    }
                }
            }
        });
    }
}

// --------------------------------------------------------------- generic

// Any radii (anisotropic boxes, radii beyond the fast kernels): direct
// extremum over the element, skipping offsets outside the volume (equal to
// the reflect boundary for these elements).  Grayscale: both extrema are
// kept as order keys; a single op returns the minimum (sign < 0: erosion)
// or the maximum.  Binary: the dilation of the (possibly complemented) bits.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void morph_generic_kernel(ChunkArgs a, Out2 o2, int se, int rz, int ry, int rx,
                                                            int both, float sign, int binary, float thr,
                                                            int use_thr, uint32_t flip)
{
    const int64_t ez = a.out_e[0], ey = a.out_e[1], ex = a.out_e[2];
    const int64_t total = ez * ey * ex;
    const Tin *in = static_cast<const Tin *>(a.in);
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = id % ex, y = (id / ex) % ey, z = id / (ex * ey);
        const int64_t gz = a.out_o[0] + z, gy = a.out_o[1] + y, gx = a.out_o[2] + x;
        int mx = INT32_MIN, mn = INT32_MAX;  // order keys (the centre voxel is always taken)
        for (int dz = -rz; dz <= rz; ++dz) {
            const int64_t zz = gz + dz;
            if (zz < 0 || zz >= a.n[0]) continue;
            for (int dy = -ry; dy <= ry; ++dy) {
                const int64_t yy = gy + dy;
                if (yy < 0 || yy >= a.n[1]) continue;
                for (int dx = -rx; dx <= rx; ++dx) {
                    const int64_t xx = gx + dx;
                    if (xx < 0 || xx >= a.n[2]) continue;
                    if (se == HARPIA_SE_BALL && dz * dz + dy * dy + dx * dx > rz * rz) continue;
                    const Tin raw = in[(zz - a.in_o[0]) * a.in_sz + (yy - a.in_o[1]) * a.in_sy + (xx - a.in_o[2])];
                    const float v = binary ? (float)(binarise(raw, thr, use_thr) ^ flip) : to_f32(raw);
                    const int k = order_key(v);
                    mx = max(mx, k);
                    mn = min(mn, k);
                }
            }
        }
        Tout *op = static_cast<Tout *>(a.out) + z * a.out_sz + y * a.out_sy + x;
        if (both) {
            *op = from_f32<Tout>(order_value(mn));
            static_cast<Tout *>(o2.ptr)[z * o2.sz + y * o2.sy + x] = from_f32<Tout>(order_value(mx));
        } else if (binary) {
            *op = from_f32<Tout>((float)((uint32_t)order_value(mx) ^ flip));
        } else {
            // grayscale single op: the minimum for an erosion (sign < 0)
            *op = from_f32<Tout>(order_value(sign < 0.f ? mn : mx));
        }
    }
}

}  // namespace morph_detail

namespace morph_detail {

template <typename T, int SE, int R, bool BOTH>
void launch_bits(const ChunkArgs &a, const MorphSpec &m, const Out2 &o2, float thr_f, hipStream_t s)
{
    static const int64_t cap = resident_blocks(bits_kernel<T, SE, R, BOTH>, kBNT);
    Tile t;
    // the kernel generation is part of the key: z splits tuned for other
    // kernels do not carry over
    const bool tuned = tune_lookup(TF_BINARY, tune_key_volume(TF_BINARY, R * 4 + SE * 2 + (BOTH ? 1 : 0),
                                                              tune_type_code<T>() + 16, a.out_e),
                                   t);
    const Grid g = make_grid(a, 4 * kBX, bits_rows<R>(), R, cap, tuned ? t.tz : 0);
    // Widest aligned access: input rows in 16-byte pieces (1- and 2-byte
    // types), else groups of 4 or 2 elements (a chain's intermediate region
    // can start 2 voxels off); output rows of 16 or 4 bytes.
    auto in_al = [&](int64_t e) {
        return ((uintptr_t)a.in % (e * sizeof(T)) == 0) && a.in_sy % e == 0 && a.in_sz % e == 0 &&
               (a.out_o[2] - a.in_o[2]) % e == 0;
    };
    const int vec_in = (sizeof(T) <= 2 && in_al(16 / (int64_t)sizeof(T))) ? 16 : (in_al(4) ? 4 : (in_al(2) ? 2 : 1));
    auto out_al = [&](int64_t e) {
        bool ok = ((uintptr_t)a.out % e == 0) && a.out_sy % e == 0 && a.out_sz % e == 0;
        if (BOTH) ok = ok && ((uintptr_t)o2.ptr % e == 0) && o2.sy % e == 0 && o2.sz % e == 0;
        return ok;
    };
    const int vec_out = out_al(16) ? 16 : (out_al(4) ? 4 : 1);
    hipLaunchKernelGGL((bits_kernel<T, SE, R, BOTH>), dim3((uint32_t)g.blocks), dim3(kBNT), 0, s, a, o2,
                       (uint32_t)(m.op == 0 ? 1u : 0u), thr_f, (int)m.has_threshold, vec_in, vec_out, g.tiles_x,
                       g.tiles_y, g.zlen);
}

// The binary kernels of one input type (every element, radius and output
// form): a function of its own, so that they compile in their own unit.
template <typename T>
bool bits_run(int r, int se, bool both, const ChunkArgs &a, const MorphSpec &m, const Out2 &o2, float thr_f,
              hipStream_t s)
{
#define HARPIA_BITS(SE_, BOTH_)                                                     \
    switch (r) {                                                                    \
    case 1: launch_bits<T, SE_, 1, BOTH_>(a, m, o2, thr_f, s); return true;         \
    case 2: launch_bits<T, SE_, 2, BOTH_>(a, m, o2, thr_f, s); return true;         \
    case 3: launch_bits<T, SE_, 3, BOTH_>(a, m, o2, thr_f, s); return true;         \
    case 4: launch_bits<T, SE_, 4, BOTH_>(a, m, o2, thr_f, s); return true;         \
    default: return false;                                                          \
    }
    if (se == HARPIA_SE_BOX) {
        if (both) { HARPIA_BITS(HARPIA_SE_BOX, true) }
        HARPIA_BITS(HARPIA_SE_BOX, false)
    }
    if (both) { HARPIA_BITS(HARPIA_SE_BALL, true) }
    HARPIA_BITS(HARPIA_SE_BALL, false)
#undef HARPIA_BITS
}

template <typename T, int SE, int R, bool BOTH>
void launch_fast(const ChunkArgs &a, const MorphSpec &m, const Out2 &o2, float thr_f, hipStream_t s)
{
    if (m.binary) {
        bits_run<T>(R, SE, BOTH, a, m, o2, thr_f, s);
    } else {
        static const int64_t cap = resident_blocks(gray_kernel<T, SE, R, BOTH>, gray_nt(R));
        Tile t;
        const bool tuned = tune_lookup(
            TF_GRAY, tune_key_volume(TF_GRAY, R * 4 + SE * 2 + (BOTH ? 1 : 0), tune_type_code<T>(), a.out_e), t);
        const Grid g = make_grid(a, gray_tx(R), kGTY, R, cap, tuned ? t.tz : 0);
        hipLaunchKernelGGL((gray_kernel<T, SE, R, BOTH>), dim3((uint32_t)g.blocks), dim3(gray_nt(R)), 0, s, a, o2,
                           m.op == 0 ? -1.f : 1.f, g.tiles_x, g.tiles_y, g.zlen);
    }
}

template <typename T, int SE, bool BOTH>
bool dispatch_r(int r, const ChunkArgs &a, const MorphSpec &m, const Out2 &o2, float thr_f, hipStream_t s)
{
    switch (r) {
    case 1: launch_fast<T, SE, 1, BOTH>(a, m, o2, thr_f, s); return true;
    case 2: launch_fast<T, SE, 2, BOTH>(a, m, o2, thr_f, s); return true;
    case 3: launch_fast<T, SE, 3, BOTH>(a, m, o2, thr_f, s); return true;
    case 4: launch_fast<T, SE, 4, BOTH>(a, m, o2, thr_f, s); return true;
    default: return false;
    }
}

template <typename T>
bool run(const ChunkArgs &a, const MorphSpec &m, bool both, const Region *out2, float thr_f, hipStream_t s)
{
    if (a.out_e[0] <= 0 || a.out_e[1] <= 0 || a.out_e[2] <= 0) return true;
    Out2 o2{nullptr, 0, 0};
    if (out2) {
        o2.ptr = out2->ptr;
        o2.sy = out2->sy;
        o2.sz = out2->sz;
    }
    const bool iso = m.r[0] == m.r[1] && m.r[1] == m.r[2];
    const bool small_slice = a.in_sy * (a.n[1] + 1) < ((int64_t)1 << 31);
    if (iso && m.r[0] >= 1 && m.r[0] <= kMaxFastR && small_slice) {
        if (m.se == HARPIA_SE_BOX)
            return both ? dispatch_r<T, HARPIA_SE_BOX, true>(m.r[0], a, m, o2, thr_f, s)
                        : dispatch_r<T, HARPIA_SE_BOX, false>(m.r[0], a, m, o2, thr_f, s);
        return both ? dispatch_r<T, HARPIA_SE_BALL, true>(m.r[0], a, m, o2, thr_f, s)
                    : dispatch_r<T, HARPIA_SE_BALL, false>(m.r[0], a, m, o2, thr_f, s);
    }
    const int64_t total = a.out_e[0] * a.out_e[1] * a.out_e[2];
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    const float sign = (!both && m.op == 0) ? -1.f : 1.f;
    const uint32_t flip = (m.binary && !both && m.op == 0) ? 1u : 0u;
    if (m.binary)
        hipLaunchKernelGGL((morph_generic_kernel<T, uint8_t>), dim3((uint32_t)blocks), dim3(256), 0, s, a, o2, m.se,
                           m.r[0], m.r[1], m.r[2], (int)both, 1.f, 1, thr_f, (int)m.has_threshold, flip);
    else
        hipLaunchKernelGGL((morph_generic_kernel<T, T>), dim3((uint32_t)blocks), dim3(256), 0, s, a, o2, m.se,
                           m.r[0], m.r[1], m.r[2], (int)both, sign, 0, thr_f, 0, 0u);
    return true;
}

}  // namespace morph_detail

template <typename T>
bool morph_run(const ChunkArgs &a, const MorphSpec &m, bool both, const Region *out2, float thr_f, hipStream_t s)
{
    return morph_detail::run<T>(a, m, both, out2, thr_f, s);
}

namespace morph_detail {

template <typename T, int SE, int R, bool BOTH>
void launch_gray_batched(BatchDesc d, float sign, hipStream_t s)
{
    static const int64_t cap = resident_blocks(gray_batched_kernel<T, SE, R, BOTH>, kGNT);
    Tile t;
    const bool tuned = tune_lookup(
        TF_GRAY_BATCHED, tune_key_batch(TF_GRAY_BATCHED, R * 4 + SE * 2 + (BOTH ? 1 : 0), tune_type_code<T>(), d), t);
    batch_layout(d, kGTX, kGTY, tuned && t.tz > 0 ? t.tz : 32);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < 8192 ? cap : 8192);
    if (grid > 0)
        hipLaunchKernelGGL((gray_batched_kernel<T, SE, R, BOTH>), dim3((uint32_t)grid), dim3(kGNT), 0, s, d, sign);
}

template <typename T, int SE, bool BOTH>
bool gray_batched_r(int r, const BatchDesc &d, float sign, hipStream_t s)
{
    switch (r) {
    case 1: launch_gray_batched<T, SE, 1, BOTH>(d, sign, s); return true;
    case 2: launch_gray_batched<T, SE, 2, BOTH>(d, sign, s); return true;
    case 3: launch_gray_batched<T, SE, 3, BOTH>(d, sign, s); return true;
    case 4: launch_gray_batched<T, SE, 4, BOTH>(d, sign, s); return true;
    default: return false;
    }
}

}  // namespace morph_detail

// Grayscale batched erosion (op 0) / dilation (op 1), or both (aux = dilation).
template <typename T>
bool morph_batched_run(const BatchDesc &d, int op, int se, int r, bool both, hipStream_t s)
{
    using namespace morph_detail;
    const float sign = (!both && op == 0) ? -1.f : 1.f;
    if (se == HARPIA_SE_BOX)
        return both ? gray_batched_r<T, HARPIA_SE_BOX, true>(r, d, sign, s)
                    : gray_batched_r<T, HARPIA_SE_BOX, false>(r, d, sign, s);
    return both ? gray_batched_r<T, HARPIA_SE_BALL, true>(r, d, sign, s)
                : gray_batched_r<T, HARPIA_SE_BALL, false>(r, d, sign, s);
}

}  // namespace harpia
