// Adjoint kernels: the sigma-gradient reduction and the subgradient of
// erosion / dilation.
//
// Morphology: erosion (dilation) is piecewise the selection of one input
// voxel per output, so its gradient routes each output's upstream gradient
// to the voxel that supplied the extremum.  Ties are broken by taking the
// first extremum in lexicographic (dz, dy, dx) order over the offsets of the
// element that fall inside the volume (a later offset wins only when it is
// strictly better).  Two kernels:
//   argext: code[p] = index of the chosen offset in the element's bounding
//           box, (dz + rz) (2ry + 1) (2rx + 1) + (dy + ry) (2rx + 1) + dx + rx;
//   gather: gin[j] = sum over offsets o of the element, in lexicographic
//           order, of g[j - o] where code[j - o] names o.
// Both stage a halo-padded 3D tile in LDS.  The gather is a deterministic
// sum in a fixed order (no atomics).
//
// sigma-gradient: per-block FP32 partials (from the fused Gaussian's dot
// epilogue, or from dot_partials_kernel) are reduced in FP64 in a fixed
// order by reduce_partials_f64.
#include <cmath>

#include "common.h"
#include "batch.h"

namespace harpia {

namespace {

constexpr int kGT = 256;            // threads
constexpr int kGX = 32, kGY = 8, kGZ = 4;  // output tile; thread = (y, x), 4 z outputs

__global__ __launch_bounds__(256) void reduce_partials_f64(const float *partials, int64_t n, double *out,
                                                           int accumulate)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)partials[i];
    sh[threadIdx.x] = s;
    lds_barrier();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        lds_barrier();
    }
    if (threadIdx.x == 0) out[0] = accumulate ? out[0] + sh[0] : sh[0];
}

// Per-block FP32 partials of sum a[p] * b[p] over a region (both strided).
__global__ __launch_bounds__(256) void dot_partials_kernel(const float *a, int64_t a_sy, int64_t a_sz,
                                                           const float *b, int64_t b_sy, int64_t b_sz, int64_t ez,
                                                           int64_t ey, int64_t ex, float *partials)
{
    const int64_t total = ez * ey * ex;
    float s = 0.f;
    for (int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x; id < total; id += (int64_t)gridDim.x * 256) {
        const int64_t x = id % ex, y = (id / ex) % ey, z = id / (ex * ey);
        s = fmaf(a[z * a_sz + y * a_sy + x], b[z * b_sz + y * b_sy + x], s);
    }
    __shared__ float wsum[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    lds_barrier();
    if (threadIdx.x == 0) partials[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

struct TileGeom {
    int64_t z0, y0, x0;  // global origin of the output tile
    int hz, hy, hx;      // LDS tile extent (tile + 2r)
};

__device__ __forceinline__ void block_tile(int tiles_x, int tiles_y, int &bx, int &by, int &bz)
{
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    bx = (int)(b % (uint32_t)tiles_x);
    by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    bz = (int)(b / (uint32_t)(tiles_x * tiles_y));
}

__device__ __forceinline__ TileGeom tile_geom(const ChunkArgs &a, int rz, int ry, int rx, int bx, int by, int bz)
{
    TileGeom t;
    t.x0 = a.out_o[2] + (int64_t)bx * kGX;
    t.y0 = a.out_o[1] + (int64_t)by * kGY;
    t.z0 = a.out_o[0] + (int64_t)bz * kGZ;
    t.hz = kGZ + 2 * rz;
    t.hy = kGY + 2 * ry;
    t.hx = kGX + 2 * rx;
    return t;
}

__device__ __forceinline__ bool in_element(int se, int r, int dz, int dy, int dx)
{
    return se == HARPIA_SE_BOX || dz * dz + dy * dy + dx * dx <= r * r;
}

// code[p] for every p of the output region (codes laid out like a.out, u16).
template <typename T>
__device__ __forceinline__ void argext_tile(const ChunkArgs &a, uint16_t *code, int op, int se, int rz, int ry,
                                            int rx, int bx, int by, int bz, float *sv)
{
    const TileGeom t = tile_geom(a, rz, ry, rx, bx, by, bz);
    const int n_lds = t.hz * t.hy * t.hx;
    const T *in = static_cast<const T *>(a.in);
    // stage the tile; positions outside the volume are clamped (never read:
    // the offset loop skips them explicitly)
    for (int e = threadIdx.x; e < n_lds; e += kGT) {
        const int lx = e % t.hx, ly = (e / t.hx) % t.hy, lz = e / (t.hx * t.hy);
        int64_t gz = t.z0 - rz + lz, gy = t.y0 - ry + ly, gx = t.x0 - rx + lx;
        gz = gz < 0 ? 0 : (gz >= a.n[0] ? a.n[0] - 1 : gz);
        gy = gy < 0 ? 0 : (gy >= a.n[1] ? a.n[1] - 1 : gy);
        gx = gx < 0 ? 0 : (gx >= a.n[2] ? a.n[2] - 1 : gx);
        // keep inside the input region as well (it covers the element's reach)
        gz = gz < a.in_o[0] ? a.in_o[0] : gz;
        gy = gy < a.in_o[1] ? a.in_o[1] : gy;
        gx = gx < a.in_o[2] ? a.in_o[2] : gx;
        sv[e] = to_f32(in[(gz - a.in_o[0]) * a.in_sz + (gy - a.in_o[1]) * a.in_sy + (gx - a.in_o[2])]);
    }
    lds_barrier();
    const int tx = threadIdx.x % kGX, ty = threadIdx.x / kGX;
    const int64_t gx = t.x0 + tx, gy = t.y0 + ty;
    const int64_t xend = a.out_o[2] + a.out_e[2], yend = a.out_o[1] + a.out_e[1];
    const int64_t zend = a.out_o[0] + a.out_e[0];
    const bool active = gx < xend && gy < yend;
    const int wx = 2 * rx + 1, wyx = (2 * ry + 1) * wx;
    for (int tz = 0; active && tz < kGZ; ++tz) {
        const int64_t gz = t.z0 + tz;
        if (gz >= zend) break;
        float best = 0.f;
        int best_code = -1;
        for (int dz = -rz; dz <= rz; ++dz) {
            if (gz + dz < 0 || gz + dz >= a.n[0]) continue;
            for (int dy = -ry; dy <= ry; ++dy) {
                if (gy + dy < 0 || gy + dy >= a.n[1]) continue;
                const float *row = sv + ((tz + rz + dz) * t.hy + (ty + ry + dy)) * t.hx + (tx + rx);
                for (int dx = -rx; dx <= rx; ++dx) {
                    if (gx + dx < 0 || gx + dx >= a.n[2]) continue;
                    if (!in_element(se, rz, dz, dy, dx)) continue;
                    const float v = row[dx];
                    const bool better = best_code < 0 || (op == HARPIA_DILATE ? v > best : v < best);
                    if (better) {
                        best = v;
                        best_code = (dz + rz) * wyx + (dy + ry) * wx + (dx + rx);
                    }
                }
            }
        }
        code[(gz - a.out_o[0]) * a.out_sz + (gy - a.out_o[1]) * a.out_sy + (gx - a.out_o[2])] =
            (uint16_t)best_code;
    }
}

template <typename T>
__global__ __launch_bounds__(kGT) void argext_kernel(ChunkArgs a, uint16_t *code, int op, int se, int rz, int ry,
                                                     int rx, int tiles_x, int tiles_y)
{
    extern __shared__ float sv[];
    int bx, by, bz;
    block_tile(tiles_x, tiles_y, bx, by, bz);
    argext_tile<T>(a, code, op, se, rz, ry, rx, bx, by, bz, sv);
}

// Batched: in = volume, aux = code volume (written).
template <typename T>
__global__ __launch_bounds__(kGT) void argext_batched_kernel(BatchDesc d, int op, int se, int rz, int ry, int rx)
{
    extern __shared__ float sv[];
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const ChunkArgs a = crop_args(d.c[c]);
        argext_tile<T>(a, static_cast<uint16_t *>(const_cast<void *>(d.c[c].aux)), op, se, rz, ry, rx, bx, by, bz,
                       sv);
        lds_barrier();
    }
}

// gin over the output region of `a` (gin laid out like a.out); g and code
// laid out like the input region of `a` (a.in describes them: in = g).
__device__ __forceinline__ void gather_tile(const ChunkArgs &a, const uint16_t *code, int se, int rz, int ry, int rx,
                                            int bx, int by, int bz, float *sg)
{
    const TileGeom t = tile_geom(a, rz, ry, rx, bx, by, bz);
    const int n_lds = t.hz * t.hy * t.hx;
    uint32_t *sc = reinterpret_cast<uint32_t *>(sg + n_lds);
    const float *g = static_cast<const float *>(a.in);
    for (int e = threadIdx.x; e < n_lds; e += kGT) {
        const int lx = e % t.hx, ly = (e / t.hx) % t.hy, lz = e / (t.hx * t.hy);
        int64_t gz = t.z0 - rz + lz, gy = t.y0 - ry + ly, gx = t.x0 - rx + lx;
        const bool inside = gz >= 0 && gz < a.n[0] && gy >= 0 && gy < a.n[1] && gx >= 0 && gx < a.n[2];
        gz = gz < 0 ? 0 : (gz >= a.n[0] ? a.n[0] - 1 : gz);
        gy = gy < 0 ? 0 : (gy >= a.n[1] ? a.n[1] - 1 : gy);
        gx = gx < 0 ? 0 : (gx >= a.n[2] ? a.n[2] - 1 : gx);
        gz = gz < a.in_o[0] ? a.in_o[0] : gz;
        gy = gy < a.in_o[1] ? a.in_o[1] : gy;
        gx = gx < a.in_o[2] ? a.in_o[2] : gx;
        const int64_t off = (gz - a.in_o[0]) * a.in_sz + (gy - a.in_o[1]) * a.in_sy + (gx - a.in_o[2]);
        sg[e] = g[off];
        sc[e] = inside ? (uint32_t)code[off] : 0xffffffffu;
    }
    lds_barrier();
    const int tx = threadIdx.x % kGX, ty = threadIdx.x / kGX;
    const int64_t gx = t.x0 + tx, gy = t.y0 + ty;
    const int64_t xend = a.out_o[2] + a.out_e[2], yend = a.out_o[1] + a.out_e[1];
    const int64_t zend = a.out_o[0] + a.out_e[0];
    const bool active = gx < xend && gy < yend;
    const int wx = 2 * rx + 1, wyx = (2 * ry + 1) * wx;
    float *gin = static_cast<float *>(a.out);
    for (int tz = 0; active && tz < kGZ; ++tz) {
        const int64_t gz = t.z0 + tz;
        if (gz >= zend) break;
        float sum = 0.f;
        for (int dz = -rz; dz <= rz; ++dz)
            for (int dy = -ry; dy <= ry; ++dy)
                for (int dx = -rx; dx <= rx; ++dx) {
                    if (!in_element(se, rz, dz, dy, dx)) continue;
                    // output p = j - o chose offset o?
                    const int e = ((tz + rz - dz) * t.hy + (ty + ry - dy)) * t.hx + (tx + rx - dx);
                    if (sc[e] == (uint32_t)((dz + rz) * wyx + (dy + ry) * wx + (dx + rx))) sum += sg[e];
                }
        gin[(gz - a.out_o[0]) * a.out_sz + (gy - a.out_o[1]) * a.out_sy + (gx - a.out_o[2])] = sum;
    }
}

__global__ __launch_bounds__(kGT) void gather_kernel(ChunkArgs a, const uint16_t *code, int se, int rz, int ry,
                                                     int rx, int tiles_x, int tiles_y)
{
    extern __shared__ float sg[];
    int bx, by, bz;
    block_tile(tiles_x, tiles_y, bx, by, bz);
    gather_tile(a, code, se, rz, ry, rx, bx, by, bz, sg);
}

// Batched: in = upstream gradient, aux = codes, out = grad_in.
__global__ __launch_bounds__(kGT) void gather_batched_kernel(BatchDesc d, int se, int rz, int ry, int rx)
{
    extern __shared__ float sg[];
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const ChunkArgs a = crop_args(d.c[c]);
        gather_tile(a, static_cast<const uint16_t *>(d.c[c].aux), se, rz, ry, rx, bx, by, bz, sg);
        lds_barrier();
    }
}

int64_t tiles_of(const ChunkArgs &a, int &tiles_x, int &tiles_y)
{
    tiles_x = (int)((a.out_e[2] + kGX - 1) / kGX);
    tiles_y = (int)((a.out_e[1] + kGY - 1) / kGY);
    return (int64_t)tiles_x * tiles_y * ((a.out_e[0] + kGZ - 1) / kGZ);
}

}  // namespace

constexpr int kMaxGradRadius = 8;

bool morph_grad_supported(const int r[3]) { return r[0] <= kMaxGradRadius && r[1] <= kMaxGradRadius && r[2] <= kMaxGradRadius; }

bool launch_argext(const ChunkArgs &a, harpia_dtype t, int op, int se, const int r[3], uint16_t *code, hipStream_t s)
{
    if (!morph_grad_supported(r)) return false;
    int tx, ty;
    const int64_t blocks = tiles_of(a, tx, ty);
    if (blocks == 0) return true;
    const size_t lds = sizeof(float) * (kGZ + 2 * r[0]) * (kGY + 2 * r[1]) * (kGX + 2 * r[2]);
#define HARPIA_ARG(DT, T)                                                                                     \
    if (t == DT) {                                                                                            \
        hipLaunchKernelGGL((argext_kernel<T>), dim3((uint32_t)blocks), dim3(kGT), lds, s, a, code, op, se, r[0], \
                           r[1], r[2], tx, ty);                                                               \
        return true;                                                                                          \
    }
    HARPIA_ARG(HARPIA_F32, float)
    HARPIA_ARG(HARPIA_U16, uint16_t)
    HARPIA_ARG(HARPIA_U8, uint8_t)
    HARPIA_ARG(HARPIA_F16, _Float16)
    HARPIA_ARG(HARPIA_BF16, bf16_t)
#undef HARPIA_ARG
    return false;
}

bool launch_gather(const ChunkArgs &a, const uint16_t *code, int se, const int r[3], hipStream_t s)
{
    if (!morph_grad_supported(r)) return false;
    int tx, ty;
    const int64_t blocks = tiles_of(a, tx, ty);
    if (blocks == 0) return true;
    const size_t lds = 8 * (size_t)(kGZ + 2 * r[0]) * (kGY + 2 * r[1]) * (kGX + 2 * r[2]);
    hipLaunchKernelGGL(gather_kernel, dim3((uint32_t)blocks), dim3(kGT), lds, s, a, code, se, r[0], r[1], r[2], tx,
                       ty);
    return true;
}

bool launch_argext_batched(const BatchDesc &d0, harpia_dtype t, int op, int se, const int r[3], hipStream_t s)
{
    if (!morph_grad_supported(r) || t != HARPIA_F32) return false;
    BatchDesc d = d0;
    batch_layout(d, kGX, kGY, kGZ);
    const size_t lds = sizeof(float) * (kGZ + 2 * r[0]) * (kGY + 2 * r[1]) * (kGX + 2 * r[2]);
    const int64_t cap = resident_blocks(argext_batched_kernel<float>, kGT, lds);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < 8192 ? cap : 8192);
    if (grid > 0)
        hipLaunchKernelGGL((argext_batched_kernel<float>), dim3((uint32_t)grid), dim3(kGT), lds, s, d, op, se, r[0],
                           r[1], r[2]);
    return true;
}

bool launch_gather_batched(const BatchDesc &d0, int se, const int r[3], hipStream_t s)
{
    if (!morph_grad_supported(r)) return false;
    BatchDesc d = d0;
    batch_layout(d, kGX, kGY, kGZ);
    const size_t lds = 8 * (size_t)(kGZ + 2 * r[0]) * (kGY + 2 * r[1]) * (kGX + 2 * r[2]);
    const int64_t cap = resident_blocks(gather_batched_kernel, kGT, lds);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < 8192 ? cap : 8192);
    if (grid > 0)
        hipLaunchKernelGGL(gather_batched_kernel, dim3((uint32_t)grid), dim3(kGT), lds, s, d, se, r[0], r[1], r[2]);
    return true;
}

void launch_reduce_f64(const float *partials, int64_t n, double *out, bool accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_partials_f64, dim3(1), dim3(256), 0, s, partials, n, out, accumulate ? 1 : 0);
}

int64_t launch_dot_partials(const Region &a, const Region &b, float *partials, int64_t max_blocks, hipStream_t s)
{
    const int64_t total = a.e[0] * a.e[1] * a.e[2];
    int64_t blocks = (total + 255) / 256;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(dot_partials_kernel, dim3((uint32_t)blocks), dim3(256), 0, s,
                       static_cast<const float *>(a.ptr), a.sy, a.sz, static_cast<const float *>(b.ptr), b.sy, b.sz,
                       a.e[0], a.e[1], a.e[2], partials);
    return blocks;
}

}  // namespace harpia
