// Sobel / Prewitt gradient magnitude (Section III-C, edge enhancement of
// the filtering suite):
//   G_a = (central difference [-1, 0, 1] along axis a) (x) (smoothing
//         [1, 2, 1] Sobel, [1, 1, 1] Prewitt, along the two other axes),
//   out = sqrt(G_z^2 + G_y^2 + G_x^2), reflect boundary.
//
// One z-streaming launch: a 512-thread workgroup owns a 128 x 16 tile of
// output columns.  Per input slice it stages the 130 x 18 patch in LDS
// (double-buffered, reflection applied to the load addresses; the next
// slice is loaded into registers while the current one is filtered), and
// each thread forms, for its 4 columns, the three in-plane responses
//   A = S_y S_x v,  B = D_y S_x v,  C = S_y D_x v.
// A 3-slice register ring then gives
//   G_z[s] = A[s+1] - A[s-1],  G_y[s] = (S_z B)[s],  G_x[s] = (S_z C)[s].
// HBM traffic is one read and one write per voxel.
#include <cmath>
#include <type_traits>

#include "common.h"

namespace harpia {
namespace edge_detail {

// Four consecutive outputs: one non-temporal 16-byte store when all 4 are
// inside the region and aligned (f32 output; the kernel never reads it
// back), else element by element.
template <typename Tout>
__device__ __forceinline__ void put4(Tout *p, const float v[4], int nvalid)
{
    if constexpr (std::is_same<Tout, float>::value) {
        if (nvalid == 4 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f q = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(q, reinterpret_cast<v4f *>(p));
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < nvalid) p[c] = from_f32<Tout>(v[c]);
}

constexpr int kNT = 512;
constexpr int kTX = 128, kTY = 16;  // one 4-column quad per thread
constexpr int PW = kTX + 2, PH = kTY + 2;
constexpr int PWP = (PW + 3) & ~3;  // 16-byte rows
constexpr int PSZ = PH * PWP;
constexpr int NLD = (PW * PH + kNT - 1) / kNT;

template <bool PREWITT>
__device__ __forceinline__ float smooth3(float a, float b, float c)
{
    return PREWITT ? (a + b) + c : fmaf(2.f, b, a + c);
}

template <typename Tin, typename Tout, bool PREWITT>
__global__ __launch_bounds__(kNT) void edge_kernel(ChunkArgs a, int zlen, int tiles_x, int tiles_y)
{
    __shared__ __attribute__((aligned(16))) float sP[2 * PSZ];

    const uint32_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % (uint32_t)tiles_x), by = (int)((blk / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(blk / (uint32_t)(tiles_x * tiles_y));
    const int tid = threadIdx.x;
    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * kTX, y0 = ybeg + (int64_t)by * kTY;
    const int64_t zo0 = a.out_o[0] + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, a.out_o[0] + a.out_e[0]);
    if (zo0 >= zo1) return;

    // in-plane source offsets and LDS slots of this thread's patch elements
    int32_t off[NLD], lds[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * kNT;
        off[i] = 0;
        lds[i] = 0;
        if (e < PW * PH) {
            const int row = e / PW, col = e - row * PW;
            int64_t gy = y0 - 1 + row;
            gy = gy > yend ? yend : gy;  // rows past the region feed no stored output
            int64_t gx = x0 - 1 + col;
            gx = gx > xend ? xend : gx;
            off[i] = (int32_t)((reflect_index(gy, a.n[1]) - a.in_o[1]) * a.in_sy +
                               (reflect_index(gx, a.n[2]) - a.in_o[2]));
            lds[i] = row * PWP + col;
        }
    }
    const Tin *in = static_cast<const Tin *>(a.in);
    const int nsteps = (int)(zo1 - zo0) + 2;  // input slices zo0 - 1 .. zo1 (reflected)
    Tin pf[NLD];
    auto fetch = [&](int j) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const Tin *base = in + (reflect_index(zo0 - 1 + j, a.n[0]) - a.in_o[0]) * a.in_sz;
#pragma unroll
        for (int i = 0; i < NLD; ++i)
            if (i < NLD - 1 || tid + i * kNT < PW * PH) pf[i] = base[off[i]];
    };

    const int qrow = tid / (kTX / 4), qcol = (tid % (kTX / 4)) * 4;
    const int64_t gy_out = y0 + qrow, gx_out = x0 + qcol;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)4, xend - gx_out) : 0;
    Tout *outp = static_cast<Tout *>(a.out) + (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);

    // ring: in-plane responses of the last three slices (slot j mod 3)
    float rA[3][4], rB[3][4], rC[3][4];

    fetch(0);
    for (int base = 0; base < nsteps; base += 3) {
        static_for<3>([&](auto U) {
            constexpr int u = decltype(U)::value;
            const int j = base + u;
            if (j >= nsteps) return;
            float *buf = sP + (j & 1) * PSZ;
#pragma unroll
            for (int i = 0; i < NLD; ++i)
                if (i < NLD - 1 || tid + i * kNT < PW * PH) buf[lds[i]] = to_f32(pf[i]);
            fetch(j + 1);
            lds_barrier();
            // in-plane responses of slice j at columns qcol .. qcol + 3
            float sx[3][4], dx[3][4];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float *row = buf + (qrow + r) * PWP + qcol;
                const float4 lo = *reinterpret_cast<const float4 *>(row);
                const float2 hi = *reinterpret_cast<const float2 *>(row + 4);
                const float v[6] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    sx[r][c] = smooth3<PREWITT>(v[c], v[c + 1], v[c + 2]);
                    dx[r][c] = v[c + 2] - v[c];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rA[u][c] = smooth3<PREWITT>(sx[0][c], sx[1][c], sx[2][c]);
                rB[u][c] = sx[2][c] - sx[0][c];
                rC[u][c] = smooth3<PREWITT>(dx[0][c], dx[1][c], dx[2][c]);
            }
            // output slice zo0 + j - 2 from slices j - 2, j - 1, j
            if (j >= 2 && nvalid > 0) {
                constexpr int s0 = (u + 1) % 3, s1 = (u + 2) % 3, s2 = u;
                const int64_t zl = zo0 + j - 2 - a.out_o[0];
                float m[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float gz = rA[s2][c] - rA[s0][c];
                    const float gy = smooth3<PREWITT>(rB[s0][c], rB[s1][c], rB[s2][c]);
                    const float gx = smooth3<PREWITT>(rC[s0][c], rC[s1][c], rC[s2][c]);
                    m[c] = sqrtf(fmaf(gz, gz, fmaf(gy, gy, gx * gx)));
                }
                put4(outp + zl * a.out_sz, m, nvalid);
            }
        });
    }
}

template <typename Tin, typename Tout>
bool run(const ChunkArgs &a, int kind, hipStream_t s)
{
    if (a.in_sy * (a.n[1] + 1) >= ((int64_t)1 << 31)) return false;  // in-plane offsets are 32-bit
    const int tiles_x = (int)((a.out_e[2] + kTX - 1) / kTX), tiles_y = (int)((a.out_e[1] + kTY - 1) / kTY);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    auto kern = kind == HARPIA_EDGE_PREWITT ? edge_kernel<Tin, Tout, true> : edge_kernel<Tin, Tout, false>;
    static const int64_t cap = resident_blocks(edge_kernel<Tin, Tout, false>, kNT);
    const int64_t nzc = z_ranges(a.out_e[0], tiles, cap, 1, 64);
    const int zlen = (int)((a.out_e[0] + nzc - 1) / nzc);
    const int64_t blocks = tiles * ((a.out_e[0] + zlen - 1) / zlen);
    hipLaunchKernelGGL(kern, dim3((uint32_t)blocks), dim3(kNT), 0, s, a, zlen, tiles_x, tiles_y);
    return true;
}

}  // namespace edge_detail

bool launch_edge(const ChunkArgs &a, harpia_dtype in_t, harpia_dtype out_t, int kind, hipStream_t s)
{
    if (a.out_e[0] <= 0 || a.out_e[1] <= 0 || a.out_e[2] <= 0) return true;
    using namespace edge_detail;
#define HARPIA_PAIR(IT, OT, TI, TO) \
    if (in_t == IT && out_t == OT) return run<TI, TO>(a, kind, s);
    HARPIA_PAIR(HARPIA_F32, HARPIA_F32, float, float)
    HARPIA_PAIR(HARPIA_U16, HARPIA_F32, uint16_t, float)
    HARPIA_PAIR(HARPIA_U8, HARPIA_F32, uint8_t, float)
    HARPIA_PAIR(HARPIA_F16, HARPIA_F16, _Float16, _Float16)
    HARPIA_PAIR(HARPIA_F16, HARPIA_F32, _Float16, float)
    HARPIA_PAIR(HARPIA_BF16, HARPIA_BF16, bf16_t, bf16_t)
    HARPIA_PAIR(HARPIA_BF16, HARPIA_F32, bf16_t, float)
#undef HARPIA_PAIR
    return false;
}

}  // namespace harpia
