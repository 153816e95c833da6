// Hessian of the Gaussian-smoothed volume in two z-streaming passes of three
// components each (texture features of the filtering suite, Section III-C),
// instead of one pass per component.
//
// Component ab is the separable correlation with, per axis, the taps of the
// derivative order that axis takes: G (order 0), D1 (order 1, odd: c_{-k} =
// -c_k, c_0 = 0) or D2 (order 2).  The two groups share their y filters and
// x inputs:
//   group 0: zz = D2_z G_y G_x,  zy = D1_z D1_y G_x,  zx = D1_z G_y D1_x
//            (y planes G, D1; three x filters; z taps D2, D1, D1)
//   group 1: yy = G_z D2_y G_x,  yx = G_z D1_y D1_x,  xx = G_z G_y D2_x
//            (y planes D2, D1, G; three x filters; z taps G)
// Per input slice a workgroup stages the (TX + 2r) x (16 + 2r) patch in LDS,
// forms the y planes from one read of each patch column, the three x-filtered
// channels, and pushes them into three register rings of 2r + 1 partial sums
// (the fused Gaussian's z pass, once per channel).  Each pass reads the
// input once and writes three volumes; the arithmetic of every channel is
// the same sequence of operations as the single-component pass, so the
// results are bitwise those of the six one-component launches.
#pragma once

#include "gauss_impl.h"

namespace harpia {
namespace gauss_detail {

constexpr int kHessMaxR = 4;  // three rings of 2r + 1 partial sums x 4 columns
constexpr int kHessTX = 128;
constexpr int kHessNT = kHessTX / 4 * kTY;

// Half taps per axis of the three derivative orders (FP64 -> FP32).
struct HessTaps {
    float g[3][kHessMaxR + 1];
    float d1[3][kHessMaxR + 1];
    float d2[3][kHessMaxR + 1];
};

// Even taps: w0 v0 + sum w_k (v_{-k} + v_k); odd: sum w_k (v_k - v_{-k}).
template <int R, bool ODD>
__device__ __forceinline__ float tap_sum(const float *v, const float *w)
{
    float s;
    if constexpr (ODD) {
        s = 0.f;
#pragma unroll
        for (int k = 1; k <= R; ++k) s = fmaf(w[k], v[R + k] - v[R - k], s);
    } else {
        s = w[0] * v[R];
#pragma unroll
        for (int k = 1; k <= R; ++k) s = fmaf(w[k], v[R - k] + v[R + k], s);
    }
    return s;
}

// Channel c of group G: its y plane (index into the group's planes), the
// order of its x and z taps.
template <int GROUP>
struct HessGroup;

template <>
struct HessGroup<0> {
    static constexpr int NY = 2;                       // y planes: G, D1
    static constexpr int yord[NY] = {0, 1};
    static constexpr int plane[3] = {0, 1, 0};         // zz: G_y, zy: D1_y, zx: G_y
    static constexpr int xord[3] = {0, 0, 1};
    static constexpr int zord[3] = {2, 1, 1};
};

template <>
struct HessGroup<1> {
    static constexpr int NY = 3;                       // y planes: D2, D1, G
    static constexpr int yord[NY] = {2, 1, 0};
    static constexpr int plane[3] = {0, 1, 2};         // yy: D2_y, yx: D1_y, xx: G_y
    static constexpr int xord[3] = {0, 1, 2};
    static constexpr int zord[3] = {0, 0, 0};
};

template <typename Tin, int R, int GROUP>
__global__ __launch_bounds__(kHessNT) void hess3_kernel(ChunkArgs a, HessTaps taps, int64_t cstride, int zlen,
                                                        int tiles_x, int tiles_y)
{
    using HG = HessGroup<GROUP>;
    constexpr int TX = kHessTX, NT = kHessNT, NY = HG::NY;
    constexpr int P = 2 * R + 1;
    constexpr int PW = TX + 2 * R;
    constexpr int PH = kTY + 2 * R;
    constexpr int PSZ = PW * PH;
    constexpr int NLD = (PSZ + NT - 1) / NT;
    constexpr int QP = (PW + 3) & ~3;
    constexpr int NYI = PW * (kTY / kMY);
    constexpr int NH = 4 + 2 * R;
    constexpr int NH4 = (NH + 3) / 4;
    constexpr int QSZ = kTY * QP + 4 * NH4;

    __shared__ float sP[2 * PSZ];
    __shared__ __attribute__((aligned(16))) float sQ[2 * NY * QSZ];

    int bx, by, bz;
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    tile_of_block(b, tiles_x, tiles_y, bx, by, bz);
    const int tid = threadIdx.x;
    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * TX;
    const int64_t y0 = ybeg + (int64_t)by * kTY;
    const int64_t zo0 = a.out_o[0] + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, a.out_o[0] + a.out_e[0]);
    if (zo0 >= zo1) return;

    // taps of each order per axis
    auto ord_taps = [&](int ord, int ax, int k) __attribute__((always_inline)) {
        return ord == 0 ? taps.g[ax][k] : (ord == 1 ? taps.d1[ax][k] : taps.d2[ax][k]);
    };
    float wy[NY][R + 1], wx[3][R + 1], wz[3][R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) {
#pragma unroll
        for (int p = 0; p < NY; ++p) wy[p][k] = ord_taps(HG::yord[p], 1, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            wx[c][k] = ord_taps(HG::xord[c], 2, k);
            wz[c][k] = ord_taps(HG::zord[c], 0, k);
        }
    }

    int32_t off[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * NT;
        off[i] = 0;
        if (e < PSZ) {
            const int row = e / PW, col = e - (e / PW) * PW;
            int64_t gy = y0 - R + row;
            gy = gy < ybeg - R ? ybeg - R : (gy > yend - 1 + R ? yend - 1 + R : gy);
            int64_t gx = x0 - R + col;
            gx = gx < xbeg - R ? xbeg - R : (gx > xend - 1 + R ? xend - 1 + R : gx);
            const int64_t ly = reflect_index(gy, a.n[1]) - a.in_o[1];
            const int64_t lx = reflect_index(gx, a.n[2]) - a.in_o[2];
            off[i] = (int32_t)(ly * a.in_sy + lx);
        }
    }

    const Tin *in = static_cast<const Tin *>(a.in);
    const int64_t s0 = zo0 - R;
    const int nsteps = (int)(zo1 - zo0) + 2 * R;
    Tin pf[NLD];
    auto fetch = [&](int j) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const Tin *base = in + (reflect_index(s0 + j, a.n[0]) - a.in_o[0]) * a.in_sz;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * NT < PSZ) pf[k] = base[off[k]];
    };
    auto stage = [&](int j) __attribute__((always_inline)) {
        float *dst = sP + (j & 1) * PSZ;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * NT < PSZ) dst[tid + k * NT] = to_f32(pf[k]);
    };

    const int qrow = tid / (TX / 4);
    const int qcol = (tid % (TX / 4)) * 4;
    const int64_t gy_out = y0 + qrow;
    const int64_t gx_out = x0 + qcol;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)4, xend - gx_out) : 0;
    float *outp = static_cast<float *>(a.out) + (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);
    const int ytid = (tid + (int)(b & 3u) * 64) & (NT - 1);

    float acc[3][P][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[c][j][q] = 0.f;

    fetch(0);
    stage(0);
    fetch(1);
    lds_barrier();

    for (int base = 0; base <= nsteps; base += P) {
        static_for<P>([&](auto UU) {
            constexpr int u = decltype(UU)::value;
            const int i = base + u;
            if (i > nsteps) return;
            if (i >= 1) {
                // x passes of slice i - 1, then its z pass; one y plane at
                // a time (its channels share the plane's row)
                const float *q = sQ + ((i - 1) & 1) * NY * QSZ;
                static_for<NY>([&](auto PPI) {
                    constexpr int p = decltype(PPI)::value;
                    float h[NH4 * 4];
                    const float4 *q4 = reinterpret_cast<const float4 *>(q + p * QSZ + qrow * QP + qcol);
#pragma unroll
                    for (int j = 0; j < NH4; ++j) {
                        const float4 t4 = q4[j];
                        h[4 * j + 0] = t4.x;
                        h[4 * j + 1] = t4.y;
                        h[4 * j + 2] = t4.z;
                        h[4 * j + 3] = t4.w;
                    }
                    static_for<3>([&](auto CC) {
                        constexpr int c = decltype(CC)::value;
                        if constexpr (HG::plane[c] == p) {
                            constexpr bool xodd = HG::xord[c] == 1, zodd = HG::zord[c] == 1;
                            float t[4];
#pragma unroll
                            for (int q4 = 0; q4 < 4; ++q4) t[q4] = tap_sum<R, xodd>(&h[q4], wx[c]);
                            static_for<P>([&](auto DD) {
                                constexpr int d = decltype(DD)::value - R;
                                constexpr int sl = (u - 1 + d + 2 * P) % P;
                                const float wd = zodd ? (d == 0 ? 0.f : (d < 0 ? wz[c][-d] : -wz[c][d]))
                                                      : wz[c][d < 0 ? -d : d];
#pragma unroll
                                for (int q4 = 0; q4 < 4; ++q4)
                                    acc[c][sl][q4] = (d == R) ? wd * t[q4] : fmaf(wd, t[q4], acc[c][sl][q4]);
                            });
                        }
                    });
                });
            }
            if (i < nsteps) {
                // y planes of slice i from one read of each patch column
                const float *pp = sP + (i & 1) * PSZ;
                float *q = sQ + (i & 1) * NY * QSZ;
#pragma unroll
                for (int itk = 0; itk < (NYI + NT - 1) / NT; ++itk) {
                    const int it = ytid + itk * NT;
                    if (itk == (NYI + NT - 1) / NT - 1 && it >= NYI) continue;
                    const int col = it % PW, rg = it / PW;
                    float v[kMY + 2 * R];
#pragma unroll
                    for (int j = 0; j < kMY + 2 * R; ++j) v[j] = pp[(rg * kMY + j) * PW + col];
                    static_for<NY>([&](auto PPI) {
                        constexpr int pl = decltype(PPI)::value;
#pragma unroll
                        for (int m = 0; m < kMY; ++m)
                            q[pl * QSZ + (rg * kMY + m) * QP + col] =
                                tap_sum<R, HG::yord[pl] == 1>(&v[m], wy[pl]);
                    });
                }
                stage(i + 1);
                fetch(i + 2);
            }
            if (i >= 1 && i - 1 >= 2 * R && nvalid > 0) {
                constexpr int sl = (u - 1 - R + 2 * P) % P;
                const int64_t o = s0 + (i - 1) - R;
                float *op = outp + (o - a.out_o[0]) * a.out_sz;
#pragma unroll
                for (int c = 0; c < 3; ++c) store4(op + c * cstride, acc[c][sl], nvalid);
            }
            if (i < nsteps) lds_barrier();
        });
    }
}

template <typename Tin, int R, int GROUP>
void launch_hess3(const ChunkArgs &a, const HessTaps &taps, int64_t cstride, hipStream_t s)
{
    static const int64_t cap = resident_blocks(hess3_kernel<Tin, R, GROUP>, kHessNT);
    const FusedGrid g = fused_grid(a, R, cap, 0, kHessTX);
    hipLaunchKernelGGL((hess3_kernel<Tin, R, GROUP>), dim3((uint32_t)g.blocks), dim3(kHessNT), 0, s, a, taps,
                       cstride, g.zlen, g.tiles_x, g.tiles_y);
}

}  // namespace gauss_detail

// The six Hessian components of a dense region in two passes (components
// zz, zy, zx, then yy, yx, xx at out, out + cstride, ... out + 5 cstride);
// equal radii 1..kHessMaxR.  false: no kernel for this radius.
template <typename Tin>
bool hess_run(const ChunkArgs &a, const gauss_detail::HessTaps &taps, int r, int64_t cstride, hipStream_t s)
{
    using namespace gauss_detail;
    ChunkArgs b = a;
    b.out = static_cast<float *>(a.out) + 3 * cstride;
    switch (r) {
#define HARPIA_CASE(RR)                                   \
    case RR:                                              \
        launch_hess3<Tin, RR, 0>(a, taps, cstride, s);    \
        launch_hess3<Tin, RR, 1>(b, taps, cstride, s);    \
        return true;
        HARPIA_CASE(1)
        HARPIA_CASE(2)
        HARPIA_CASE(3)
        HARPIA_CASE(4)
#undef HARPIA_CASE
    default:
        return false;
    }
}

}  // namespace harpia
