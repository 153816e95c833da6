// Otsu's global threshold (Section III-C, threshold algorithms of the label
// editing module) for integer volumes, one histogram bin per value:
//   1. histogram, privatised per workgroup in LDS: u8 with one 256-bin copy
//      per wave; u16 with 32768 32-bit bins per workgroup, so each segment
//      of the volume is read by two workgroups, one per half of the value
//      range (neighbours on one XCD, so the second read mostly hits L2);
//      the LDS bins are then added to 64-bit global bins;
//   2. one workgroup scans the counts and the value-weighted counts and
//      picks the split k (class 0: values <= k) maximising the between-class
//      variance w0 w1 (m0 - m1)^2 -- in FP64, in a fixed order, from exact
//      integer sums, so the argmax is decided as the FP64 definition decides
//      it; the first maximum wins;
//   3. out = (v > k) as uint8, k read from device memory (no host round
//      trip between the three launches).
// Volumes stream through 16-byte loads; a misaligned head or a tail is read
// element by element.
#include "common.h"

namespace harpia {
namespace otsu_detail {

constexpr int kNT = 256;
constexpr int kHistNT = 1024;
constexpr int kScanNT = 1024;
constexpr int kHalf = 32768;  // u16 bins per workgroup

// Calls f(value) for every element of the 16-byte vector q of T.
template <typename T, class F>
__device__ __forceinline__ void each_value(const uint4 &q, F &f)
{
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if constexpr (sizeof(T) == 1) {
#pragma unroll
            for (int b = 0; b < 4; ++b) f((w[j] >> (8 * b)) & 0xffu);
        } else {
            f(w[j] & 0xffffu);
            f(w[j] >> 16);
        }
    }
}

// Calls f(value) for every element of v[lo, hi), spread over the workgroup.
template <typename T, class F>
__device__ __forceinline__ void each_in_range(const T *v, int64_t lo, int64_t hi, F &f)
{
    constexpr int V = 16 / (int)sizeof(T);
    constexpr int U = 4;  // vectors in flight per thread
    const int tid = threadIdx.x;
    const int64_t mis = (int64_t)(((uintptr_t)(v + lo) & 15) / sizeof(T));
    const int64_t head = mis ? min(hi - lo, (int64_t)V - mis) : 0;
    for (int64_t i = lo + tid; i < lo + head; i += kHistNT) f((uint32_t)v[i]);
    const int64_t a = lo + head;
    const int64_t nvec = (hi - a) / V;
    const uint4 *p = reinterpret_cast<const uint4 *>(v + a);
    int64_t i = tid;
    for (; i + (U - 1) * kHistNT < nvec; i += U * kHistNT) {
        uint4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = p[i + u * kHistNT];
#pragma unroll
        for (int u = 0; u < U; ++u) each_value<T>(q[u], f);
    }
    for (; i < nvec; i += kHistNT) {
        const uint4 q = p[i];
        each_value<T>(q, f);
    }
    for (int64_t e = a + nvec * V + tid; e < hi; e += kHistNT) f((uint32_t)v[e]);
}

// u8: workgroup b counts v[b per, (b + 1) per) into one LDS copy per wave.
__global__ __launch_bounds__(kHistNT) void hist8_kernel(const uint8_t *v, int64_t n, int64_t per,
                                                        unsigned long long *hist)
{
    constexpr int W = kHistNT / 64;
    __shared__ uint32_t sh[W * 256];
    for (int i = threadIdx.x; i < W * 256; i += kHistNT) sh[i] = 0;
    lds_barrier();
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(n, lo + per);
    uint32_t *mine = sh + (threadIdx.x / 64) * 256;
    auto count = [&](uint32_t x) __attribute__((always_inline)) { atomicAdd(&mine[x], 1u); };
    if (lo < hi) each_in_range<uint8_t>(v, lo, hi, count);
    lds_barrier();
    if (threadIdx.x < 256) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) c += sh[w * 256 + threadIdx.x];
        if (c) atomicAdd(&hist[threadIdx.x], (unsigned long long)c);
    }
}

// u16: logical workgroup b counts the values of half (b & 1) of the range
// in segment b >> 1.
__global__ __launch_bounds__(kHistNT) void hist16_kernel(const uint16_t *v, int64_t n, int64_t per,
                                                         unsigned long long *hist)
{
    __shared__ uint32_t sh[kHalf];
    for (int i = threadIdx.x; i < kHalf; i += kHistNT) sh[i] = 0;
    lds_barrier();
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t half = b & 1u;
    const int64_t lo = (int64_t)(b >> 1) * per, hi = min(n, lo + per);
    auto count = [&](uint32_t x) __attribute__((always_inline)) {
        if ((x >> 15) == half) atomicAdd(&sh[x & (kHalf - 1)], 1u);
    };
    if (lo < hi) each_in_range<uint16_t>(v, lo, hi, count);
    lds_barrier();
    for (int i = threadIdx.x; i < kHalf; i += kHistNT) {
        const uint32_t c = sh[i];
        if (c) atomicAdd(&hist[half * kHalf + i], (unsigned long long)c);
    }
}

// Between-class variance of the split with c0 voxels (value sum s0) below,
// out of n (value sum total); the same operations in the same order as the
// FP64 definition, without contraction.
__device__ __forceinline__ double between(unsigned long long c0, unsigned long long s0, unsigned long long n,
                                          unsigned long long total)
{
#pragma clang fp contract(off)
    const unsigned long long c1 = n - c0;
    const double d = (double)s0 / (double)c0 - (double)(total - s0) / (double)c1;
    return ((double)c0 * (double)c1) * (d * d);
}

template <int NB>
__global__ __launch_bounds__(kScanNT) void scan_kernel(const unsigned long long *hist, int64_t *result)
{
    constexpr int PER = (NB + kScanNT - 1) / kScanNT;
    __shared__ unsigned long long sc[kScanNT], ss[kScanNT];
    __shared__ double sb[kScanNT];
    __shared__ int sk[kScanNT];
    const int t = threadIdx.x;
    unsigned long long c = 0, s = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int k = t * PER + j;
        if (k < NB) {
            c += hist[k];
            s += (unsigned long long)k * hist[k];
        }
    }
    sc[t] = c;
    ss[t] = s;
    lds_barrier();
    // inclusive scan over the thread chunks (exact integer sums)
    for (int off = 1; off < kScanNT; off <<= 1) {
        const unsigned long long ac = t >= off ? sc[t - off] : 0, as = t >= off ? ss[t - off] : 0;
        lds_barrier();
        sc[t] += ac;
        ss[t] += as;
        lds_barrier();
    }
    const unsigned long long n = sc[kScanNT - 1], total = ss[kScanNT - 1];
    unsigned long long c0 = sc[t] - c, s0 = ss[t] - s;  // before this thread's chunk
    double best = -1.0;
    int best_k = -1;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int k = t * PER + j;
        if (k < NB - 1) {
            c0 += hist[k];
            s0 += (unsigned long long)k * hist[k];
            if (c0 != 0 && c0 != n) {
                const double b = between(c0, s0, n, total);
                if (b > best) {
                    best = b;
                    best_k = k;
                }
            }
        }
    }
    sb[t] = best;
    sk[t] = best_k;
    lds_barrier();
    // argmax, ties to the smaller k (k = -1: no split in that chunk)
    for (int w = kScanNT / 2; w > 0; w >>= 1) {
        if (t < w) {
            const double ob = sb[t + w];
            const int ok = sk[t + w];
            const bool take = ok >= 0 && (sk[t] < 0 || ob > sb[t] || (ob == sb[t] && ok < sk[t]));
            if (take) {
                sb[t] = ob;
                sk[t] = ok;
            }
        }
        lds_barrier();
    }
    if (t == 0) result[0] = sk[0];
}

// out = (v > k): 16 elements per thread and step through 16-byte loads and
// stores when both pointers are 16-byte aligned (vec), else one element.
template <typename T>
__global__ __launch_bounds__(kNT) void binarize_kernel(const T *v, int64_t n, const int64_t *k, uint8_t *out,
                                                       int vec)
{
    const int64_t kk = k[0];
    const int64_t stride = (int64_t)gridDim.x * kNT;
    const int64_t id = (int64_t)blockIdx.x * kNT + threadIdx.x;
    int64_t done = 0;
    if (vec) {
        const int64_t nv = n / 16;
        const uint4 *p = reinterpret_cast<const uint4 *>(v);
        uint4 *o = reinterpret_cast<uint4 *>(out);
        for (int64_t i = id; i < nv; i += stride) {
            uint32_t r[4] = {0, 0, 0, 0};
            int m = 0;
            auto put = [&](uint32_t x) __attribute__((always_inline)) {
                r[m >> 2] |= ((int64_t)x > kk ? 1u : 0u) << (8 * (m & 3));
                ++m;
            };
            if constexpr (sizeof(T) == 1) {
                const uint4 q = p[i];
                each_value<T>(q, put);
            } else {
                const uint4 q0 = p[2 * i], q1 = p[2 * i + 1];
                each_value<T>(q0, put);
                each_value<T>(q1, put);
            }
            o[i] = make_uint4(r[0], r[1], r[2], r[3]);
        }
        done = nv * 16;
    }
    for (int64_t i = done + id; i < n; i += stride) out[i] = (int64_t)v[i] > kk ? 1 : 0;
}

// Segment length of the histogram: a multiple of 64 elements (so every
// segment starts 16-byte aligned when the volume does).
inline int64_t segment(int64_t n, int64_t segs)
{
    int64_t per = (n + segs - 1) / segs;
    return (per + 63) / 64 * 64;
}

template <typename T>
void run(const T *v, int64_t n, uint8_t *out, unsigned long long *hist, int64_t *result, hipStream_t s)
{
    constexpr int NB = sizeof(T) == 1 ? 256 : 65536;
    if constexpr (sizeof(T) == 1) {
        static const int64_t cap = resident_blocks(hist8_kernel, kHistNT);
        const int64_t per = segment(n, cap);
        const int64_t blocks = (n + per - 1) / per;
        hipLaunchKernelGGL(hist8_kernel, dim3((uint32_t)blocks), dim3(kHistNT), 0, s, v, n, per, hist);
    } else {
        static const int64_t cap = resident_blocks(hist16_kernel, kHistNT);
        const int64_t segs = cap / 2 > 0 ? cap / 2 : 1;
        const int64_t per = segment(n, segs);
        const int64_t blocks = 2 * ((n + per - 1) / per);
        hipLaunchKernelGGL(hist16_kernel, dim3((uint32_t)blocks), dim3(kHistNT), 0, s, v, n, per, hist);
    }
    hipLaunchKernelGGL((scan_kernel<NB>), dim3(1), dim3(kScanNT), 0, s, hist, result);
    if (out) {
        static const int64_t cap_b = resident_blocks(binarize_kernel<T>, kNT);
        const int vec = (((uintptr_t)v | (uintptr_t)out) & 15) == 0;
        int64_t bb = (n / (vec ? 16 : 1) + kNT - 1) / kNT;
        if (bb > 4 * cap_b) bb = 4 * cap_b;
        if (bb < 1) bb = 1;
        hipLaunchKernelGGL((binarize_kernel<T>), dim3((uint32_t)bb), dim3(kNT), 0, s, v, n, result, out, vec);
    }
}

}  // namespace otsu_detail

int otsu_bins(harpia_dtype t) { return t == HARPIA_U8 ? 256 : (t == HARPIA_U16 ? 65536 : 0); }

bool launch_otsu(const void *v, harpia_dtype t, int64_t n, uint8_t *out, unsigned long long *hist, int64_t *result,
                 hipStream_t s)
{
    if (t == HARPIA_U8)
        otsu_detail::run<uint8_t>(static_cast<const uint8_t *>(v), n, out, hist, result, s);
    else if (t == HARPIA_U16)
        otsu_detail::run<uint16_t>(static_cast<const uint16_t *>(v), n, out, hist, result, s);
    else
        return false;
    return true;
}

}  // namespace harpia
