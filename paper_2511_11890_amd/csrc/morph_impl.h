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
// f32 and all u8/u16/f16/bf16 values are f32 values).  Binary erosion is the
// complement of the dilation of the complement.  "Both" kernels return the
// erosion and the dilation from one read of the input.
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
// Binary data is packed 4 voxels per 32-bit word (one byte each, 0 or 1):
// extrema become AND / OR on words and x shifts are byte funnel shifts.
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

    // Double-buffered patch: slice i is staged into sP[i & 1] while other
    // threads may still read slice i - 1 from the other half, so one barrier
    // per slice suffices.  Every thread derives the x-runs it needs straight
    // from the patch (no intermediate LDS arrays).
    __shared__ __attribute__((aligned(16))) float sP[2 * BUF];

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

    float acc[NM][P][kGC];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < kGC; ++c) acc[m][j][c] = 0.f;

    fetch(0);

    // Step i (0 .. nsteps): stage slice i and fetch slice i + 1, store the
    // output completed by step i - 1 (after the fetch, so that the next
    // staging waits only for work issued a step earlier), then filter slice i.
    for (int base = 0; base <= nsteps; base += P) {
        static_for<P>([&](auto U) {
            constexpr int u = decltype(U)::value;
            const int i = base + u;
            if (i > nsteps) return;
            float *buf = sP + (i & 1) * BUF;
            if (i < nsteps) {
#pragma unroll
                for (int k = 0; k < NLD; ++k)
                    if (k < NLD - 1 || tid + k * NT < PSZ)
                        buf[lds[k]] = BOTH ? to_f32(pf[k]) : sign * to_f32(pf[k]);
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
                            outp[zl * a.out_sz + q] = from_f32<T>(acc[1][sl][q]);
                            outp2[zl * o2.sz + q] = from_f32<T>(acc[0][sl][q]);
                        }
                } else {
#pragma unroll
                    for (int q = 0; q < kGC; ++q)
                        if (q < nvalid) outp[zl * a.out_sz + q] = from_f32<T>(sign * acc[0][sl][q]);
                }
            }
            if (i >= nsteps) return;
            lds_barrier();

            // In-plane disc of every z-class (kGC columns): rows dy = -R .. R,
            // each row's x-runs of the half-widths its classes take.
            float disc[NM][S::NC][kGC];
            static_for<P>([&](auto DY) {
                constexpr int dy = decltype(DY)::value - R;
                constexpr int hmax = S::max_hw(dy);
                if constexpr (hmax >= 0) {
                    float v[NV4 * 4];
                    const float *prow = &buf[(qrow + R + dy) * PWP + qcol];
                    if constexpr (kGC % 4 == 0) {
                        const float4 *p4 = reinterpret_cast<const float4 *>(prow);
#pragma unroll
                        for (int j = 0; j < NV4; ++j) {
                            const float4 t4 = p4[j];
                            v[4 * j] = t4.x;
                            v[4 * j + 1] = t4.y;
                            v[4 * j + 2] = t4.z;
                            v[4 * j + 3] = t4.w;
                        }
                    } else {
                        const float2 *p2 = reinterpret_cast<const float2 *>(prow);
#pragma unroll
                        for (int j = 0; j < 2 * NV4; ++j) {
                            const float2 t2 = p2[j];
                            v[2 * j] = t2.x;
                            v[2 * j + 1] = t2.y;
                        }
                    }
#pragma unroll
                    for (int m = 0; m < NM; ++m) {
                        float run[kGC];
#pragma unroll
                        for (int q = 0; q < kGC; ++q) run[q] = v[q + R];
                        static_for<hmax + 1>([&](auto H) {
                            constexpr int h = decltype(H)::value;
                            if constexpr (h > 0) {
#pragma unroll
                                for (int q = 0; q < kGC; ++q)
                                    run[q] = (m == 0) ? fmaxf(run[q], fmaxf(v[q + R - h], v[q + R + h]))
                                                      : fminf(run[q], fminf(v[q + R - h], v[q + R + h]));
                            }
                            static_for<S::NC>([&](auto C) {
                                constexpr int c = decltype(C)::value;
                                if constexpr (S::takes(c, dy, h)) {
                                    constexpr bool first = (dy == -S::rho(c));
#pragma unroll
                                    for (int q = 0; q < kGC; ++q)
                                        disc[m][c][q] = first ? run[q]
                                                              : ((m == 0) ? fmaxf(disc[m][c][q], run[q])
                                                                          : fminf(disc[m][c][q], run[q]));
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
                                                 : ((m == 0) ? fmaxf(acc[m][sl][q], disc[m][c][q])
                                                             : fminf(acc[m][sl][q], disc[m][c][q]));
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

constexpr int kBTX = 256;             // voxels per tile row (64 words)
constexpr int kBTY = 16;
constexpr int kBW = kBTX / 4;         // words per tile row
constexpr int kBPW = kBW + 2;         // patch words per row (1 halo word a side)

__device__ __forceinline__ uint32_t funnel_bytes(uint32_t hi, uint32_t lo, int k)
{
    // bytes k..k+3 of the 8-byte little-endian value hi:lo (0 <= k <= 4)
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * k));
}

// Store 16 output bytes (4 packed words), or the first `nvalid` of them.
__device__ __forceinline__ void emit16(uint8_t *p, uint4 w, int nvalid)
{
    if (nvalid == 16 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        *reinterpret_cast<uint4 *>(p) = w;
        return;
    }
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 16; ++q)
        if (q < nvalid) p[q] = (uint8_t)((ws[q >> 2] >> (8 * (q & 3))) & 0xffu);
}

template <typename Tin>
__device__ __forceinline__ uint32_t binarise(Tin v, float thr, bool use_thr)
{
    const float f = to_f32(v);
    return use_thr ? (f > thr ? 1u : 0u) : (f != 0.f ? 1u : 0u);
}

// Binary erosion / dilation: u8 {0, 1} output.  `flip` = 1 computes an
// erosion (complement in and out), 0 a dilation; BOTH writes the erosion to
// out and the dilation to out2.
template <typename Tin, int SE, int R, bool BOTH>
__global__ __launch_bounds__(kNT) void binary_kernel(ChunkArgs a, Out2 o2, uint32_t flip, float thr, int use_thr,
                                                     int tiles_x, int tiles_y, int zlen)
{
    static_assert(R >= 1 && R <= 4, "one halo word per side");
    using S = Shape<SE, R>;
    constexpr int P = 2 * R + 1;
    constexpr int PH = kBTY + 2 * R;
    constexpr int NWI = kBPW * PH;                 // patch words
    constexpr int NLW = (NWI + kNT - 1) / kNT;     // words loaded per thread
    constexpr int NA = kBW * PH;                   // stage A items
    constexpr int NM = BOTH ? 2 : 1;               // 0: OR (dilation), 1: AND
    const uint32_t fmask = flip ? 0x01010101u : 0u;

    __shared__ uint32_t sP[PH * kBPW];
    __shared__ __attribute__((aligned(16))) uint32_t sH[NM][S::NL][PH * kBW];

    const int tid = threadIdx.x;
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(b % (uint32_t)tiles_x);
    const int by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(b / (uint32_t)(tiles_x * tiles_y));

    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * kBTX;
    const int64_t y0 = ybeg + (int64_t)by * kBTY;
    const int64_t zo0 = a.out_o[0] + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, a.out_o[0] + a.out_e[0]);
    if (zo0 >= zo1) return;

    // Each loaded word holds patch columns 4w-4 .. 4w-1 relative to x0.  Its
    // source offset is kept when the 4 voxels are consecutive in memory;
    // words that cross a face or the clamp (-1) are resolved per voxel.
    int32_t off[NLW];
#pragma unroll
    for (int i = 0; i < NLW; ++i) {
        const int e = tid + i * kNT;
        off[i] = 0;
        if (e < NWI) {
            const int row = e / kBPW, w = e - (e / kBPW) * kBPW;
            int64_t gy = y0 - R + row;
            gy = gy < ybeg - R ? ybeg - R : (gy > yend - 1 + R ? yend - 1 + R : gy);
            const int64_t ly = reflect_index(gy, a.n[1]) - a.in_o[1];
            const int64_t gx = x0 - 4 + 4 * w;
            if (gx >= 0 && gx + 3 < a.n[2] && gx >= xbeg - R && gx + 3 <= xend - 1 + R)
                off[i] = (int32_t)(ly * a.in_sy + (gx - a.in_o[2]));
            else
                off[i] = -1 - (int32_t)ly;  // slow path marker, keeps the row
        }
    }

    const int64_t s0 = zo0 - R;
    const int nsteps = (int)(zo1 - zo0) + 2 * R;
    const Tin *in = static_cast<const Tin *>(a.in);
    // The next slice, packed on load (unconditional fetch, clamped at the end).
    uint32_t pf[NLW];
    auto fetch = [&](int j) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const Tin *base = in + (reflect_index(s0 + j, a.n[0]) - a.in_o[0]) * a.in_sz;
#pragma unroll
        for (int i = 0; i < NLW; ++i) {
            if (i < NLW - 1 || tid + i * kNT < NWI) {
                uint32_t wv = 0;
                if (off[i] >= 0) {
                    const Tin *p = base + off[i];
#pragma unroll
                    for (int j = 0; j < 4; ++j) wv |= binarise(p[j], thr, use_thr) << (8 * j);
                } else {
                    const int e = tid + i * kNT;
                    const int w = e % kBPW;
                    const int64_t ly = -1 - (int64_t)off[i];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        int64_t gx = x0 - 4 + 4 * w + j;
                        gx = gx < xbeg - R ? xbeg - R : (gx > xend - 1 + R ? xend - 1 + R : gx);
                        const int64_t lx = reflect_index(gx, a.n[2]) - a.in_o[2];
                        wv |= binarise(base[ly * a.in_sy + lx], thr, use_thr) << (8 * j);
                    }
                }
                pf[i] = wv;
            }
        }
    };

    const int qrow = tid / (kBW / 4);
    const int qw = (tid % (kBW / 4)) * 4;  // first word of this thread's quad
    const int64_t gy_out = y0 + qrow;
    const int64_t gx_out = x0 + 4 * qw;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)16, xend - gx_out) : 0;
    uint8_t *outp = static_cast<uint8_t *>(a.out) + (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);
    uint8_t *outp2 = BOTH ? static_cast<uint8_t *>(o2.ptr) + (gy_out - ybeg) * o2.sy + (gx_out - xbeg) : nullptr;

    uint32_t acc[NM][P][4];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[m][j][c] = 0u;

    fetch(0);

    for (int base = 0; base <= nsteps; base += P) {
        static_for<P>([&](auto U) {
            constexpr int u = decltype(U)::value;
            const int i = base + u;
            if (i > nsteps) return;
            if (i < nsteps) {
#pragma unroll
                for (int k = 0; k < NLW; ++k)
                    if (k < NLW - 1 || tid + k * kNT < NWI) sP[tid + k * kNT] = BOTH ? pf[k] : (pf[k] ^ fmask);
                fetch(i + 1);
            }
            if (i >= 1 && i - 1 >= 2 * R && nvalid > 0) {
                constexpr int sl = (u - 1 - R + 2 * P) % P;
                const int64_t zl = s0 + (i - 1) - R - a.out_o[0];
                if constexpr (BOTH) {
                    emit16(outp + zl * a.out_sz, make_uint4(acc[1][sl][0], acc[1][sl][1], acc[1][sl][2], acc[1][sl][3]),
                           nvalid);
                    emit16(outp2 + zl * o2.sz, make_uint4(acc[0][sl][0], acc[0][sl][1], acc[0][sl][2], acc[0][sl][3]),
                           nvalid);
                } else {
                    emit16(outp + zl * a.out_sz,
                           make_uint4(acc[0][sl][0] ^ fmask, acc[0][sl][1] ^ fmask, acc[0][sl][2] ^ fmask,
                                      acc[0][sl][3] ^ fmask),
                           nvalid);
                }
            }
            if (i >= nsteps) return;
            lds_barrier();

            // stage A: word-level x runs (OR for m = 0, AND for m = 1)
#pragma unroll
            for (int itk = 0; itk < (NA + kNT - 1) / kNT; ++itk) {
                const int it = tid + itk * kNT;
                if (itk == (NA + kNT - 1) / kNT - 1 && it >= NA) continue;
                const int row = it / kBW, w = it - (it / kBW) * kBW;
                const uint32_t wl = sP[row * kBPW + w];
                const uint32_t wc = sP[row * kBPW + w + 1];
                const uint32_t wr = sP[row * kBPW + w + 2];
#pragma unroll
                for (int m = 0; m < NM; ++m) {
                    uint32_t run = wc;
                    static_for<R + 1>([&](auto H) {
                        constexpr int h = decltype(H)::value;
                        if constexpr (h > 0) {
                            const uint32_t sr = funnel_bytes(wr, wc, h);      // voxel x + h
                            const uint32_t sl2 = funnel_bytes(wc, wl, 4 - h); // voxel x - h
                            run = (m == 0) ? (run | sr | sl2) : (run & sr & sl2);
                        }
                        if constexpr (SE != HARPIA_SE_BOX || h == R) sH[m][S::lvl(h)][row * kBW + w] = run;
                    });
                }
            }
            lds_barrier();

#pragma unroll
            for (int m = 0; m < NM; ++m) {
                static_for<S::NC>([&](auto C) {
                    constexpr int c = decltype(C)::value;
                    constexpr int rh = S::rho(c);
                    uint32_t dv[4];
                    static_for<2 * rh + 1>([&](auto DY) {
                        constexpr int dy = decltype(DY)::value - rh;
                        constexpr int l = S::lvl(S::hw(c, dy));
                        const uint4 t4 = *reinterpret_cast<const uint4 *>(&sH[m][l][(qrow + R + dy) * kBW + qw]);
                        const uint32_t tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if constexpr (dy == -rh) dv[q] = tv[q];
                            else dv[q] = (m == 0) ? (dv[q] | tv[q]) : (dv[q] & tv[q]);
                        }
                    });
                    static_for<P>([&](auto DD) {
                        constexpr int d = decltype(DD)::value - R;
                        if constexpr (S::cls(d) == c) {
                            constexpr int sl = (u + d + 2 * P) % P;
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                acc[m][sl][q] = (d == R) ? dv[q]
                                                         : ((m == 0) ? (acc[m][sl][q] | dv[q])
                                                                     : (acc[m][sl][q] & dv[q]));
                        }
                    });
                });
            }
        });
    }
}

// --------------------------------------------------------------- generic

// Any radii (anisotropic boxes, radii beyond the fast kernels): direct
// extremum over the element, skipping offsets outside the volume (equal to
// the reflect boundary for these elements).  mode 0: dilation (or erosion of
// sign-flipped data), 2: both.
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
        float mx = -INFINITY, mn = INFINITY;
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
                    float v = binary ? (float)(binarise(raw, thr, use_thr) ^ flip) : sign * to_f32(raw);
                    mx = fmaxf(mx, v);
                    mn = fminf(mn, v);
                }
            }
        }
        Tout *op = static_cast<Tout *>(a.out) + z * a.out_sz + y * a.out_sy + x;
        if (both) {
            *op = from_f32<Tout>(mn);
            static_cast<Tout *>(o2.ptr)[z * o2.sz + y * o2.sy + x] = from_f32<Tout>(mx);
        } else if (binary) {
            *op = from_f32<Tout>((float)((uint32_t)mx ^ flip));
        } else {
            *op = from_f32<Tout>(sign * mx);
        }
    }
}

}  // namespace morph_detail

namespace morph_detail {

template <typename T, int SE, int R, bool BOTH>
void launch_fast(const ChunkArgs &a, const MorphSpec &m, const Out2 &o2, float thr_f, hipStream_t s)
{
    if (m.binary) {
        static const int64_t cap = resident_blocks(binary_kernel<T, SE, R, BOTH>, kNT);
        Tile t;
        const bool tuned = tune_lookup(
            TF_BINARY, tune_key_volume(TF_BINARY, R * 4 + SE * 2 + (BOTH ? 1 : 0), tune_type_code<T>(), a.out_e), t);
        const Grid g = make_grid(a, kBTX, kBTY, R, cap, tuned ? t.tz : 0);
        hipLaunchKernelGGL((binary_kernel<T, SE, R, BOTH>), dim3((uint32_t)g.blocks), dim3(kNT), 0, s, a, o2,
                           (uint32_t)(m.op == 0 ? 1u : 0u), thr_f, (int)m.has_threshold, g.tiles_x, g.tiles_y,
                           g.zlen);
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
