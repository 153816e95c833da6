// Gaussian smoothing kernels for gfx950 (the Gaussian filter of the
// library's filtering suite, Section III-C).
//
// out[z,y,x] = sum_{a,b,c} wz[a] wy[b] wx[c] in[R(z+a), R(y+b), R(x+c)]
// with half-sample reflection R and normalised sampled taps (FP64 -> FP32).
//
// Fused kernel (equal radius r on all axes, 1 <= r <= kGaussFusedMaxR):
//   one workgroup owns a TX x 16 tile of output columns (TX = 128 with 512
//   threads for r <= 6, TX = 64 with 256 threads above; one 4-column quad
//   per thread) and streams along z over a range of output slices.  Per
//   input slice it
//     1. stages the (TX+2r) x (16+2r) patch in LDS (reflection applied on
//        load, converted to f32) -- the global loads of the next slice are
//        issued before the current slice is filtered, so HBM latency hides
//        behind the LDS work;
//     2. y pass from LDS, register-blocked kMY rows per work item;
//     3. x pass from LDS, 4 adjacent columns per thread (b128 LDS reads);
//     4. z pass in registers: each thread keeps a ring of 2r+1 partial sums
//        for each of its 4 columns; slice s adds w|s-o| * t to output o for
//        o in [s-r, s+r], and output s-r is then complete and stored.
//   HBM traffic is one read of the input and one write of the output per
//   voxel (halo re-reads hit L2: xcd_remap keeps neighbouring tiles on one
//   XCD).  The ring is indexed statically by unrolling the slice loop 2r+1
//   times.
//
// Unfused kernels (any radius up to kMaxGaussRadius, anisotropic radii):
//   three 1D passes through FP32 scratch, one thread per output voxel.
#include <cmath>

#include "common.h"
#include "gauss_grid.h"
#include "batch.h"

namespace harpia {

template <typename Tin, typename Tout>
bool gauss_run(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s, void *scratch, size_t scratch_bytes);
template <typename Tin, typename Tout>
bool gauss_batched_run(const BatchDesc &d, const GaussTaps &taps, hipStream_t s);
template <typename Tin>
int64_t gauss_sigma3_run(const Tin *x, const float *g, const int64_t n[3], const GaussTaps &wt, const GaussTaps &dt,
                         hipStream_t s, float *partials);
template <typename Tin>
int64_t gauss_sigma3_batched_run(const BatchDesc &d, const GaussTaps &wt, const GaussTaps &dt, hipStream_t s,
                                 float *partials);

int64_t launch_gauss_sigma3(const void *x, harpia_dtype x_t, const float *g, const int64_t n[3], const GaussTaps &wt,
                            const GaussTaps &dt, hipStream_t s, float *partials)
{
    if (n[1] * n[2] >= ((int64_t)1 << 31)) return -1;  // in-plane offsets are 32-bit
    switch (x_t) {
    case HARPIA_F32: return gauss_sigma3_run<float>(static_cast<const float *>(x), g, n, wt, dt, s, partials);
    case HARPIA_U16: return gauss_sigma3_run<uint16_t>(static_cast<const uint16_t *>(x), g, n, wt, dt, s, partials);
    case HARPIA_U8: return gauss_sigma3_run<uint8_t>(static_cast<const uint8_t *>(x), g, n, wt, dt, s, partials);
    case HARPIA_F16: return gauss_sigma3_run<_Float16>(static_cast<const _Float16 *>(x), g, n, wt, dt, s, partials);
    case HARPIA_BF16: return gauss_sigma3_run<bf16_t>(static_cast<const bf16_t *>(x), g, n, wt, dt, s, partials);
    }
    return -1;
}

int64_t gauss_sigma3_blocks_bound(const int64_t n[3])
{
    const int64_t tiles = ((n[2] + gauss_detail::kTX - 1) / gauss_detail::kTX) *
                          ((n[1] + gauss_detail::kTY - 1) / gauss_detail::kTY);
    return tiles * (n[0] < gauss_detail::kMaxZRanges ? n[0] : gauss_detail::kMaxZRanges);
}

int64_t launch_gauss_sigma3_batched(const BatchDesc &d, const GaussTaps &wt, const GaussTaps &dt, hipStream_t s,
                                    float *partials)
{
    return gauss_sigma3_batched_run<float>(d, wt, dt, s, partials);
}

void make_gauss_dtaps3(const double sigma[3], const int radius[3], GaussTaps &t)
{
    make_gauss_taps_r(sigma, radius, t);
    for (int a = 0; a < 3; ++a) {
        GaussTaps one;
        make_gauss_dtaps_r(sigma, radius, a, one);
        for (int k = 0; k <= kMaxGaussRadius; ++k) t.w[a][k] = one.w[a][k];
    }
}

// Batched kernels are built for float32 volumes (the differentiable path).
bool launch_gauss_batched(const BatchDesc &d, harpia_dtype in_t, harpia_dtype out_t, const GaussTaps &taps,
                          hipStream_t s)
{
    if (in_t != HARPIA_F32 || out_t != HARPIA_F32) return false;
    return gauss_batched_run<float, float>(d, taps, s);
}

int64_t gauss_batched_max_partials() { return 8192; }

size_t gaussian_scratch_bytes(const int64_t out_e[3], const int r[3], bool fused)
{
    if (fused && r[0] == r[1] && r[1] == r[2] && r[0] >= 1 && r[0] <= kGaussFusedMaxR) return 0;
    // worst case input region: output extent + 2r per axis
    const int64_t iz = out_e[0] + 2 * r[0], iy = out_e[1] + 2 * r[1];
    return (size_t)((iz * iy * out_e[2] + iz * out_e[1] * out_e[2]) * (int64_t)sizeof(float));
}

void make_mean_taps(const int radius[3], GaussTaps &t)
{
    t.amount = 0.f;
    t.unsharp = 0;
    t.odd = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int r = radius[ax];
        t.r[ax] = r;
        const double w = 1.0 / (double)(2 * r + 1);
        for (int k = 0; k <= kMaxGaussRadius; ++k) t.w[ax][k] = (k <= r) ? (float)w : 0.f;
    }
}

void make_gauss_deriv_taps(const double sigma[3], const int radius[3], const int order[3], GaussTaps &t)
{
    t.amount = 0.f;
    t.unsharp = 0;
    t.odd = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int r = radius[ax];
        t.r[ax] = r;
        const double s2 = sigma[ax] * sigma[ax];
        double e[kMaxGaussRadius + 1];
        double total = 0.0;
        for (int k = 0; k <= r; ++k) {
            e[k] = std::exp(-((double)k * (double)k) / (2.0 * s2));
            total += (k == 0) ? e[k] : 2.0 * e[k];
        }
        for (int k = 0; k <= kMaxGaussRadius; ++k) {
            double c = 0.0;
            if (k <= r) {
                const double w = e[k] / total;
                c = order[ax] == 0 ? w : (order[ax] == 1 ? (double)k / s2 * w : ((double)k * k - s2) / (s2 * s2) * w);
            }
            t.w[ax][k] = (float)c;
        }
        if (order[ax] == 1) t.odd |= 1 << ax;
    }
}

void make_gauss_taps_r(const double sigma[3], const int radius[3], GaussTaps &t)
{
    t.amount = 0.f;
    t.unsharp = 0;
    t.odd = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int r = radius[ax];
        t.r[ax] = r;
        double e[kMaxGaussRadius + 1];
        double total = 0.0;
        for (int k = 0; k <= r; ++k) {
            e[k] = std::exp(-((double)k * (double)k) / (2.0 * sigma[ax] * sigma[ax]));
            total += (k == 0) ? e[k] : 2.0 * e[k];
        }
        for (int k = 0; k <= kMaxGaussRadius; ++k) t.w[ax][k] = (k <= r) ? (float)(e[k] / total) : 0.f;
    }
}

void make_gauss_dtaps_r(const double sigma[3], const int radius[3], int d_axis, GaussTaps &t)
{
    make_gauss_taps_r(sigma, radius, t);
    const int r = radius[d_axis];
    const double sg = sigma[d_axis];
    double e[kMaxGaussRadius + 1];
    double total = 0.0, m2 = 0.0;
    for (int k = 0; k <= r; ++k) {
        e[k] = std::exp(-((double)k * (double)k) / (2.0 * sg * sg));
        total += (k == 0) ? e[k] : 2.0 * e[k];
    }
    for (int k = 1; k <= r; ++k) m2 += 2.0 * (e[k] / total) * (double)k * (double)k;
    for (int k = 0; k <= kMaxGaussRadius; ++k)
        t.w[d_axis][k] = (k <= r) ? (float)((e[k] / total) * ((double)k * k - m2) / (sg * sg * sg)) : 0.f;
}

void make_gauss_taps(const double sigma[3], double truncate, GaussTaps &t)
{
    int r[3];
    for (int ax = 0; ax < 3; ++ax) r[ax] = (int)(truncate * sigma[ax] + 0.5);
    make_gauss_taps_r(sigma, r, t);
}

bool launch_gaussian(const ChunkArgs &a, harpia_dtype in_t, harpia_dtype out_t, const GaussTaps &taps,
                     hipStream_t s, void *scratch, size_t scratch_bytes)
{
    if (a.out_e[0] <= 0 || a.out_e[1] <= 0 || a.out_e[2] <= 0) return true;
#define HARPIA_PAIR(IT, OT, TI, TO) \
    if (in_t == IT && out_t == OT) return gauss_run<TI, TO>(a, taps, s, scratch, scratch_bytes);
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
