// Local thresholds (Section III-C, threshold algorithms of the label
// editing module): out = (v > T) as uint8 with, per voxel,
//   mean:     T = m - offset,                m the box mean (weights w),
//   gaussian: T = (G v) - offset,            the same with Gaussian weights,
//   niblack:  T = m + k s,                   s = sqrt(mean(v^2) - m^2),
//   sauvola:  T = m (1 + k (s / R - 1)).
// One z-streaming launch per chunk on the skeleton of the fused Gaussian:
// a TX x 16 tile of output columns (TX = 128 or 64, see thresh_tx), the
// (TX+2r) x (16+2r) patch staged in
// LDS per slice (the next slice loaded into registers meanwhile), y and x
// passes from LDS and a z ring of 2r+1 partial sums per column in
// registers -- one channel (the weighted mean), or two (v and v^2) for the
// standard deviation.  The centre voxel the threshold is compared with is
// read one slice ahead.  HBM traffic: the input once, one byte out.
#include <cmath>

#include "common.h"

namespace harpia {
namespace thresh_detail {

constexpr int kTY = 16, kMY = 4;
// Tile width: 128 columns (512 threads) while the register ring of 2r + 1
// slices x NCH channels stays small, else 64 columns (256 threads); one
// 4-column quad per thread.
constexpr int thresh_tx(int r, int nch) { return (2 * r + 1) * nch <= 13 ? 128 : 64; }
constexpr int thresh_nt(int r, int nch) { return thresh_tx(r, nch) / 4 * kTY; }
constexpr int kMaxR1 = 12;  // one channel
constexpr int kMaxR2 = 6;   // two channels (the ring doubles)

struct Params {
    int method;  // harpia_threshold_method
    float k, r_param, offset;
};

__device__ __forceinline__ uint8_t decide(const Params &p, float x, float m, float q)
{
    float t;
    if (p.method == HARPIA_THRESHOLD_MEAN || p.method == HARPIA_THRESHOLD_GAUSSIAN) {
        t = m - p.offset;
    } else {
        const float sd = sqrtf(fmaxf(fmaf(-m, m, q), 0.f));
        t = p.method == HARPIA_THRESHOLD_NIBLACK ? fmaf(p.k, sd, m) : m * fmaf(p.k, sd / p.r_param - 1.f, 1.f);
    }
    return x > t ? 1 : 0;
}

template <typename Tin, int R, int NCH>
__global__ __launch_bounds__(thresh_nt(R, NCH)) void thresh_kernel(ChunkArgs a, GaussTaps taps, Params prm, int zlen, int tiles_x,
                                                     int tiles_y)
{
    constexpr int TX = thresh_tx(R, NCH), NT = thresh_nt(R, NCH);
    constexpr int P = 2 * R + 1;
    constexpr int PW = TX + 2 * R, PH = kTY + 2 * R, PSZ = PW * PH;
    constexpr int NLD = (PSZ + NT - 1) / NT;
    constexpr int QP = (PW + 3) & ~3;
    constexpr int NYI = PW * (kTY / kMY);
    constexpr int NH = 4 + 2 * R, NH4 = (NH + 3) / 4;
    constexpr int QSZ = kTY * QP + 4 * NH4;

    __shared__ float sP[2 * PSZ];
    __shared__ __attribute__((aligned(16))) float sQ[NCH][2 * QSZ];

    const uint32_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(blk % (uint32_t)tiles_x), by = (int)((blk / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(blk / (uint32_t)(tiles_x * tiles_y));
    const int tid = threadIdx.x;
    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * TX, y0 = ybeg + (int64_t)by * kTY;
    const int64_t zo0 = a.out_o[0] + (int64_t)bz * zlen;
    const int64_t zo1 = min(zo0 + (int64_t)zlen, a.out_o[0] + a.out_e[0]);
    if (zo0 >= zo1) return;

    float wz[R + 1], wy[R + 1], wx[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        wz[k] = taps.w[0][k];
        wy[k] = taps.w[1][k];
        wx[k] = taps.w[2][k];
    }

    int32_t off[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * NT;
        off[i] = 0;
        if (e < PSZ) {
            const int row = e / PW, col = e - row * PW;
            int64_t gy = y0 - R + row;
            gy = gy > yend - 1 + R ? yend - 1 + R : gy;
            int64_t gx = x0 - R + col;
            gx = gx > xend - 1 + R ? xend - 1 + R : gx;
            off[i] = (int32_t)((reflect_index(gy, a.n[1]) - a.in_o[1]) * a.in_sy +
                               (reflect_index(gx, a.n[2]) - a.in_o[2]));
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

    const int qrow = tid / (TX / 4), qcol = (tid % (TX / 4)) * 4;
    const int64_t gy_out = y0 + qrow, gx_out = x0 + qcol;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)4, xend - gx_out) : 0;
    uint8_t *outp = static_cast<uint8_t *>(a.out) + (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);
    const Tin *inc = in + (gy_out - a.in_o[1]) * a.in_sy + (gx_out - a.in_o[2]);  // centre column

    float acc[NCH][P][4];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int j = 0; j < P; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[ch][j][c] = 0.f;
    Tin xc[4];  // centre voxels of the next output slice

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
                // x pass and z ring of slice i - 1, every channel
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const float4 *q4 = reinterpret_cast<const float4 *>(sQ[ch] + ((i - 1) & 1) * QSZ + qrow * QP + qcol);
                    float h[NH4 * 4];
#pragma unroll
                    for (int j = 0; j < NH4; ++j) {
                        const float4 t4 = q4[j];
                        h[4 * j] = t4.x, h[4 * j + 1] = t4.y, h[4 * j + 2] = t4.z, h[4 * j + 3] = t4.w;
                    }
                    float t[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        float sacc = wx[0] * h[c + R];
#pragma unroll
                        for (int k = 1; k <= R; ++k) sacc = fmaf(wx[k], h[c + R - k] + h[c + R + k], sacc);
                        t[c] = sacc;
                    }
                    static_for<P>([&](auto DD) {
                        constexpr int d = decltype(DD)::value - R;
                        constexpr int sl = (u - 1 + d + 2 * P) % P;
                        const float wd = wz[d < 0 ? -d : d];
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            acc[ch][sl][c] = (d == R) ? wd * t[c] : fmaf(wd, t[c], acc[ch][sl][c]);
                    });
                }
            }
            if (i < nsteps) {
                // y pass of slice i: channel 0 weights v, channel 1 v^2
                const float *p = sP + (i & 1) * PSZ;
#pragma unroll
                for (int itk = 0; itk < (NYI + NT - 1) / NT; ++itk) {
                    const int it = tid + itk * NT;
                    if (itk == (NYI + NT - 1) / NT - 1 && it >= NYI) continue;
                    const int col = it % PW, rg = it / PW;
                    float v[kMY + 2 * R];
#pragma unroll
                    for (int j = 0; j < kMY + 2 * R; ++j) v[j] = p[(rg * kMY + j) * PW + col];
#pragma unroll
                    for (int m = 0; m < kMY; ++m) {
                        float s1 = wy[0] * v[m + R];
#pragma unroll
                        for (int k = 1; k <= R; ++k) s1 = fmaf(wy[k], v[m + R - k] + v[m + R + k], s1);
                        sQ[0][(i & 1) * QSZ + (rg * kMY + m) * QP + col] = s1;
                        if constexpr (NCH == 2) {
                            float s2 = wy[0] * v[m + R] * v[m + R];
#pragma unroll
                            for (int k = 1; k <= R; ++k)
                                s2 = fmaf(wy[k], fmaf(v[m + R - k], v[m + R - k], v[m + R + k] * v[m + R + k]), s2);
                            sQ[1][(i & 1) * QSZ + (rg * kMY + m) * QP + col] = s2;
                        }
                    }
                }
                stage(i + 1);
                fetch(i + 2);
            }
            // output i - 1 - R is complete: compare its centre voxels
            if (i >= 1 && i - 1 >= 2 * R && nvalid > 0) {
                constexpr int sl = (u - 1 - R + 2 * P) % P;
                const int64_t o = s0 + (i - 1) - R;
                uint8_t b[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    b[c] = decide(prm, to_f32(xc[c]), acc[0][sl][c], NCH == 2 ? acc[NCH - 1][sl][c] : 0.f);
                uint8_t *dst = outp + (o - a.out_o[0]) * a.out_sz;
                if (nvalid == 4 && (reinterpret_cast<uintptr_t>(dst) & 3) == 0) {
                    *reinterpret_cast<uint32_t *>(dst) =
                        (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (c < nvalid) dst[c] = b[c];
                }
            }
            // the output of step i + 1 (slice s0 + i - R): load its centre voxels
            if (i - R >= R && i < nsteps && nvalid > 0) {
                const Tin *src = inc + (s0 + i - R - a.in_o[0]) * a.in_sz;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < nvalid) xc[c] = src[c];
            }
            if (i < nsteps) lds_barrier();
        });
    }
}

template <typename Tin, int R, int NCH>
void launch(const ChunkArgs &a, const GaussTaps &taps, const Params &prm, hipStream_t s)
{
    constexpr int TX = thresh_tx(R, NCH), NT = thresh_nt(R, NCH);
    static const int64_t cap = resident_blocks(thresh_kernel<Tin, R, NCH>, NT);
    const int tiles_x = (int)((a.out_e[2] + TX - 1) / TX), tiles_y = (int)((a.out_e[1] + kTY - 1) / kTY);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    const int64_t nzc = z_ranges(a.out_e[0], tiles, cap, R, 64);
    const int zlen = (int)((a.out_e[0] + nzc - 1) / nzc);
    const int64_t blocks = tiles * ((a.out_e[0] + zlen - 1) / zlen);
    hipLaunchKernelGGL((thresh_kernel<Tin, R, NCH>), dim3((uint32_t)blocks), dim3(NT), 0, s, a, taps, prm, zlen,
                       tiles_x, tiles_y);
}

template <typename Tin, int NCH>
bool dispatch(int r, const ChunkArgs &a, const GaussTaps &taps, const Params &prm, hipStream_t s)
{
    switch (r) {
#define HARPIA_CASE(RR)                                        \
    case RR:                                                   \
        if (RR > (NCH == 2 ? kMaxR2 : kMaxR1)) return false;   \
        launch<Tin, (RR > (NCH == 2 ? kMaxR2 : kMaxR1) ? 1 : RR), NCH>(a, taps, prm, s); \
        return true;
        HARPIA_CASE(1)
        HARPIA_CASE(2)
        HARPIA_CASE(3)
        HARPIA_CASE(4)
        HARPIA_CASE(5)
        HARPIA_CASE(6)
        HARPIA_CASE(7)
        HARPIA_CASE(8)
        HARPIA_CASE(9)
        HARPIA_CASE(10)
        HARPIA_CASE(11)
        HARPIA_CASE(12)
#undef HARPIA_CASE
    default:
        return false;
    }
}

template <typename Tin>
bool run(const ChunkArgs &a, const GaussTaps &taps, const Params &prm, hipStream_t s)
{
    if (!(taps.r[0] == taps.r[1] && taps.r[1] == taps.r[2])) return false;
    if (a.in_sy * (a.n[1] + 1) >= ((int64_t)1 << 31)) return false;  // in-plane offsets are 32-bit
    const bool two = prm.method == HARPIA_THRESHOLD_NIBLACK || prm.method == HARPIA_THRESHOLD_SAUVOLA;
    return two ? dispatch<Tin, 2>(taps.r[0], a, taps, prm, s) : dispatch<Tin, 1>(taps.r[0], a, taps, prm, s);
}

}  // namespace thresh_detail

int local_threshold_max_radius(int method)
{
    const bool two = method == HARPIA_THRESHOLD_NIBLACK || method == HARPIA_THRESHOLD_SAUVOLA;
    return two ? thresh_detail::kMaxR2 : thresh_detail::kMaxR1;
}

bool launch_local_threshold(const ChunkArgs &a, harpia_dtype in_t, const GaussTaps &taps, int method, float k,
                            float r_param, float offset, hipStream_t s)
{
    if (a.out_e[0] <= 0 || a.out_e[1] <= 0 || a.out_e[2] <= 0) return true;
    const thresh_detail::Params prm{method, k, r_param, offset};
    switch (in_t) {
    case HARPIA_F32: return thresh_detail::run<float>(a, taps, prm, s);
    case HARPIA_U16: return thresh_detail::run<uint16_t>(a, taps, prm, s);
    case HARPIA_U8: return thresh_detail::run<uint8_t>(a, taps, prm, s);
    default: return false;
    }
}

}  // namespace harpia
