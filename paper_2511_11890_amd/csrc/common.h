// Internal definitions shared by the HIP kernels and the host engine of
// libharpia.  Not part of the public ABI (that is include/harpia.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <cstdlib>
#include <string>

#include "harpia.h"

namespace harpia {

// ----------------------------------------------------------------- errors

struct Error {
    harpia_status status;
    std::string message;
};

[[noreturn]] void fail(harpia_status st, const std::string &msg);
void check_hip(hipError_t e, const char *what);

// ----------------------------------------------------------------- dtypes

struct bf16_t {
    uint16_t bits;
};

size_t dtype_size(harpia_dtype t);
const char *dtype_name(harpia_dtype t);

// Element conversions used inside kernels.  Every storage type converts to
// float exactly (u8, u16, f16 and bf16 values are all representable).
__device__ __forceinline__ float to_f32(uint8_t v) { return (float)v; }
__device__ __forceinline__ float to_f32(uint16_t v) { return (float)v; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16_t v)
{
    return __uint_as_float(((uint32_t)v.bits) << 16);
}

template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v)
{
    return (_Float16)v;  // round to nearest even
}
// Round to nearest even: add 0x7fff plus the lowest kept bit, truncate.
// NaN keeps its sign and becomes a quiet NaN.
template <> __device__ __forceinline__ bf16_t from_f32<bf16_t>(float v)
{
    uint32_t u = __float_as_uint(v);
    bf16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        r.bits = (uint16_t)((u >> 16) | 0x0040u);
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        r.bits = (uint16_t)(u >> 16);
    }
    return r;
}
// Morphology outputs are input values, so these conversions are exact.
template <> __device__ __forceinline__ uint16_t from_f32<uint16_t>(float v)
{
    return (uint16_t)v;
}
template <> __device__ __forceinline__ uint8_t from_f32<uint8_t>(float v)
{
    return (uint8_t)v;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also fences
// global memory, which makes every wave wait for all of its outstanding
// global loads (vmcnt(0)) at each barrier and so defeats prefetching the
// next slices; the streaming kernels exchange data through LDS only.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------ reflection

// Half-sample symmetric reflection of i into [0, n), valid for any i.
// Calls f(std::integral_constant<int, I>) for I = 0..N-1 with I a
// compile-time constant, so register arrays indexed by I stay in registers.
template <int... I, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F &&f)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(std::make_integer_sequence<int, N>{}, static_cast<F &&>(f));
}

__host__ __device__ __forceinline__ int64_t reflect_index(int64_t i, int64_t n)
{
    if (i >= 0 && i < n) return i;
    int64_t p = 2 * n;
    int64_t m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

// --------------------------------------------------------------- regions

// A box-shaped region of a volume stored densely in device memory:
// element (z, y, x) of the region (global coordinates o + (z, y, x)) lives at
// ptr + z * sz + y * sy + x (element units).
struct Region {
    void *ptr;
    int64_t sy, sz;
    int64_t o[3];  // global origin {z, y, x}
    int64_t e[3];  // extent
};

// Kernel-side description of one filter application on a chunk: read from
// `in` (which covers every reflected index the output region needs), write
// the output region `out`.  n[] is the global volume extent.
struct ChunkArgs {
    const void *in;
    int64_t in_sy, in_sz;
    int64_t in_o[3];
    void *out;
    int64_t out_sy, out_sz;
    int64_t out_o[3];
    int64_t out_e[3];
    int64_t n[3];
};

inline ChunkArgs make_chunk_args(const Region &in, const Region &out, const int64_t n[3])
{
    ChunkArgs a;
    a.in = in.ptr;
    a.in_sy = in.sy;
    a.in_sz = in.sz;
    a.out = out.ptr;
    a.out_sy = out.sy;
    a.out_sz = out.sz;
    for (int i = 0; i < 3; ++i) {
        a.in_o[i] = in.o[i];
        a.out_o[i] = out.o[i];
        a.out_e[i] = out.e[i];
        a.n[i] = n[i];
    }
    return a;
}

// Map a linear block index so that the blocks one XCD runs (the hardware
// deals consecutive workgroups round-robin over the 8 XCDs) cover a
// contiguous range of tiles, which then share halos in that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    constexpr uint32_t kXcd = 8;
    uint32_t full = nb - nb % kXcd;
    if (b >= full) return b;
    return (b % kXcd) * (full / kXcd) + b / kXcd;
}

// ------------------------------------------------------------ launchers

// Workgroups of `kernel` the whole device holds at once (occupancy per CU x
// CU count); at least 1.
template <class K>
inline int64_t resident_blocks(K kernel, int threads, size_t dyn_lds = 0)
{
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, dyn_lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1024;
    }
    return (int64_t)(nb > 0 ? nb : 1) * (cus > 0 ? cus : 1);
}

// Number of z ranges to split `nz` output slices into, for `tiles` xy tiles
// per range on a device holding `capacity` workgroups at once: minimises
// (rounds of resident workgroups) x (slices one workgroup streams, its 2r
// warm-up included), preferring fewer ranges on ties.
inline int64_t z_ranges(int64_t nz, int64_t tiles, int64_t capacity, int r, int64_t max_ranges = 64)
{
    // HARPIA_ZRANGES=n forces n ranges (a tuning knob: the same work, split
    // differently across workgroups)
    static const int64_t forced = [] {
        const char *e = std::getenv("HARPIA_ZRANGES");
        return (e && *e) ? (int64_t)std::atoll(e) : (int64_t)0;
    }();
    if (forced > 0) {
        const int64_t n = forced < nz ? forced : nz;
        return n < max_ranges ? n : max_ranges;
    }
    int64_t best_n = 1;
    double best = 1e300;
    for (int64_t zc = 1; zc <= nz && zc <= max_ranges; ++zc) {
        const int64_t zlen = (nz + zc - 1) / zc;
        const int64_t n = (nz + zlen - 1) / zlen;
        const int64_t rounds = (tiles * n + capacity - 1) / capacity;
        const double cost = (double)rounds * (double)(zlen + 2 * r);
        if (cost < best * 0.999) {
            best = cost;
            best_n = n;
        }
    }
    return best_n;
}
constexpr int kMaxGaussRadius = 64;  // unfused-path limit per axis
constexpr int kGaussFusedMaxR = 12;  // fused z-streaming kernel: 1 <= r <= this

struct GaussTaps {
    int r[3];                                 // radius per axis {z, y, x}
    float w[3][kMaxGaussRadius + 1];          // half taps w[a][|k|], FP32
    float amount;                             // unsharp mask amount a (used when unsharp != 0)
    int unsharp;                              // 1: out = (1 + a) x - a (G x); 0: out = G x
    int odd;                                  // bit a (z 1, y 2, x 4): axis a has odd taps c_{-k} = -c_k,
                                              // c_0 = 0, w[k] = c_k for k >= 1
};

// The taps a fused z-streaming kernel takes as a kernel argument (radii up
// to kGaussFusedMaxR): 160 bytes instead of GaussTaps' 804, so that a
// 64-crop batch descriptor plus two tap sets fit the 4 KiB argument space.
struct FusedTaps {
    float w[3][kGaussFusedMaxR + 1];  // half taps w[a][|k|], FP32
    float amount;                     // unsharp mask amount
};

inline FusedTaps fused_taps(const GaussTaps &t)
{
    FusedTaps f;
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k <= kGaussFusedMaxR; ++k) f.w[a][k] = t.w[a][k];
    f.amount = t.amount;
    return f;
}

// Fills taps in FP64 and rounds them to FP32 (host).
void make_gauss_taps(const double sigma[3], double truncate, GaussTaps &t);
void make_gauss_taps_r(const double sigma[3], const int radius[3], GaussTaps &t);
// Uniform taps 1 / (2 r + 1) per axis (the mean filter), in FP64 then FP32.
void make_mean_taps(const int radius[3], GaussTaps &t);
// Correlation taps of the order[a]-th derivative (0, 1, 2) of the Gaussian
// smoothing along each axis, from the FP64 normalised taps w:
// order 1: (k / s^2) w_k (odd), order 2: ((k^2 - s^2) / s^4) w_k.
void make_gauss_deriv_taps(const double sigma[3], const int radius[3], const int order[3], GaussTaps &t);
// As make_gauss_taps_r, with axis `d_axis` replaced by d w / d sigma (radius
// held fixed): w_k (k^2 - sum_j w_j j^2) / sigma^3, in FP64.
void make_gauss_dtaps_r(const double sigma[3], const int radius[3], int d_axis, GaussTaps &t);
// d w / d sigma on every axis (the D taps of the three-term sigma-gradient).
void make_gauss_dtaps3(const double sigma[3], const int radius[3], GaussTaps &t);
// The three sigma-gradient terms of a dense device volume in one pass
// (x of dtype x_t, g float32; equal radii 1..12): partials[a nb + b] for
// axis a = z, y, x; returns nb (at most gauss_sigma3_blocks_bound), or -1.
int64_t launch_gauss_sigma3(const void *x, harpia_dtype x_t, const float *g, const int64_t n[3], const GaussTaps &wt,
                            const GaussTaps &dt, hipStream_t s, float *partials);
int64_t gauss_sigma3_blocks_bound(const int64_t n[3]);
// The six Hessian components of a dense region in two three-component
// passes (out, out + cstride, ..., out + 5 cstride: zz, zy, zx, yy, yx, xx);
// float32 input, equal radii 1..4.  false: not supported (no launch).
bool launch_hessian_fused(const ChunkArgs &a, harpia_dtype in_t, const double sigma[3], const int r[3],
                          int64_t cstride, hipStream_t s);

// Launch the Gaussian on one chunk.  Returns false if no kernel handles the
// dtype pair / radius combination (caller reports UNSUPPORTED).
bool launch_gaussian(const ChunkArgs &a, harpia_dtype in_t, harpia_dtype out_t,
                     const GaussTaps &taps, hipStream_t s, void *scratch,
                     size_t scratch_bytes);
// Otsu's threshold of a device volume (u8 / u16): hist (otsu_bins(t)
// 64-bit counters, zeroed by the caller) and result (1 int64) are device
// scratch; out (may be NULL) receives v > k.  Returns false for other dtypes.
int otsu_bins(harpia_dtype t);
bool launch_otsu(const void *v, harpia_dtype t, int64_t n, uint8_t *out, unsigned long long *hist, int64_t *result,
                 hipStream_t s);
// Local threshold of one chunk (uint8 out); taps hold the box or Gaussian
// weights.  Returns false for unsupported dtypes / radii.
bool launch_local_threshold(const ChunkArgs &a, harpia_dtype in_t, const GaussTaps &taps, int method, float k,
                            float r_param, float offset, hipStream_t s);
int local_threshold_max_radius(int method);
// Sobel (kind 0) / Prewitt (kind 1) gradient magnitude of one chunk (radius
// 1 halo); dtype pairs as for the Gaussian.
bool launch_edge(const ChunkArgs &a, harpia_dtype in_t, harpia_dtype out_t, int kind, hipStream_t s);
// Scratch bytes the Gaussian needs for an output region of `out_e` voxels
// (0 for the fused kernel).
// fused = false: the bytes of the unfused passes even where a fused kernel
// exists (odd taps are fused for float32 -> float32 only).
size_t gaussian_scratch_bytes(const int64_t out_e[3], const int r[3], bool fused = true);
// The fused Gaussian addresses a slice of the input with 32-bit offsets: a
// volume of extent n whose slices are too large takes the unfused passes.
inline bool gauss_slices_fit(const int64_t n[3]) { return n[2] * (n[1] + 1) < ((int64_t)1 << 31); }

struct MorphSpec {
    int op;              // 0 erode (min), 1 dilate (max)
    int se;              // harpia_se
    int r[3];            // radius per axis
    bool binary;         // binarise on load, u8 output
    bool has_threshold;  // binary: compare with threshold; else v != 0
    double threshold;
};

bool launch_morph(const ChunkArgs &a, harpia_dtype t, const MorphSpec &m, hipStream_t s);
// With both = true the step writes the erosion to a.out and the dilation to
// *out2 from one read of the input.
bool launch_morph_ex(const ChunkArgs &a, harpia_dtype t, const MorphSpec &m, bool both, const Region *out2,
                     hipStream_t s);
float compare_threshold(harpia_dtype t, double thr);

// ---------------------------------------------------------- adjoints

// sum of partials[0..n) in FP64, fixed order, into out[0] (or added to it).
void launch_reduce_f64(const float *partials, int64_t n, double *out, bool accumulate, hipStream_t s);
// Per-block partials of sum a * b over a region; returns the block count.
int64_t launch_dot_partials(const Region &a, const Region &b, float *partials, int64_t max_blocks, hipStream_t s);
// Erosion / dilation subgradient: codes of the first extremum, then the
// gather of the upstream gradient.  Radii up to 8 per axis.
bool morph_grad_supported(int se, const int r[3]);
bool launch_argext(const ChunkArgs &a, harpia_dtype t, int op, int se, const int r[3], uint16_t *code,
                   hipStream_t s);
bool launch_gather(const ChunkArgs &a, const uint16_t *code, int se, const int r[3], hipStream_t s);

}  // namespace harpia
