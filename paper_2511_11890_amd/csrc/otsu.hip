// Otsu's global threshold (Section III-C, threshold algorithms of the label
// editing module) for integer volumes, one histogram bin per value:
//   1. histogram: u8 in per-workgroup LDS bins merged with 64-bit atomics,
//      u16 straight into 65536 global 64-bit bins (they live in L2);
//   2. one workgroup scans the counts and the value-weighted counts and
//      picks the split k (class 0: values <= k) maximising the between-class
//      variance w0 w1 (m0 - m1)^2 -- in FP64, in a fixed order, from exact
//      integer sums, so the argmax is decided as the FP64 definition decides
//      it; the first maximum wins;
//   3. out = (v > k) as uint8, k read from device memory (no host round
//      trip between the three launches).
#include "common.h"

namespace harpia {
namespace otsu_detail {

constexpr int kNT = 256;
constexpr int kScanNT = 1024;

template <typename T, int NB>
__global__ __launch_bounds__(kNT) void hist_kernel(const T *v, int64_t n, unsigned long long *hist)
{
    const int64_t stride = (int64_t)gridDim.x * kNT;
    if constexpr (NB <= 4096) {
        __shared__ uint32_t sh[NB];
        for (int i = threadIdx.x; i < NB; i += kNT) sh[i] = 0;
        lds_barrier();
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride) atomicAdd(&sh[v[i]], 1u);
        lds_barrier();
        for (int i = threadIdx.x; i < NB; i += kNT)
            if (sh[i]) atomicAdd(&hist[i], (unsigned long long)sh[i]);
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride)
            atomicAdd(&hist[v[i]], 1ull);
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

template <typename T>
__global__ __launch_bounds__(kNT) void binarize_kernel(const T *v, int64_t n, const int64_t *k, uint8_t *out)
{
    const int64_t kk = k[0];
    const int64_t stride = (int64_t)gridDim.x * kNT;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += stride)
        out[i] = (int64_t)v[i] > kk ? 1 : 0;
}

template <typename T, int NB>
void run(const T *v, int64_t n, uint8_t *out, unsigned long long *hist, int64_t *result, hipStream_t s)
{
    static const int64_t cap_h = resident_blocks(hist_kernel<T, NB>, kNT);
    int64_t blocks = (n + kNT - 1) / kNT;
    if (blocks > cap_h) blocks = cap_h;
    hipLaunchKernelGGL((hist_kernel<T, NB>), dim3((uint32_t)blocks), dim3(kNT), 0, s, v, n, hist);
    hipLaunchKernelGGL((scan_kernel<NB>), dim3(1), dim3(kScanNT), 0, s, hist, result);
    if (out) {
        static const int64_t cap_b = resident_blocks(binarize_kernel<T>, kNT);
        int64_t bb = (n + kNT - 1) / kNT;
        if (bb > 4 * cap_b) bb = 4 * cap_b;
        hipLaunchKernelGGL((binarize_kernel<T>), dim3((uint32_t)bb), dim3(kNT), 0, s, v, n, result, out);
    }
}

}  // namespace otsu_detail

int otsu_bins(harpia_dtype t) { return t == HARPIA_U8 ? 256 : (t == HARPIA_U16 ? 65536 : 0); }

bool launch_otsu(const void *v, harpia_dtype t, int64_t n, uint8_t *out, unsigned long long *hist, int64_t *result,
                 hipStream_t s)
{
    if (t == HARPIA_U8)
        otsu_detail::run<uint8_t, 256>(static_cast<const uint8_t *>(v), n, out, hist, result, s);
    else if (t == HARPIA_U16)
        otsu_detail::run<uint16_t, 65536>(static_cast<const uint16_t *>(v), n, out, hist, result, s);
    else
        return false;
    return true;
}

}  // namespace harpia
