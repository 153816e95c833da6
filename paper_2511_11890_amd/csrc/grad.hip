// Adjoint kernels: the sigma-gradient reduction and the subgradient of
// erosion / dilation.
//
// Morphology: erosion (dilation) is piecewise the selection of one input
// voxel per output, so its gradient routes each output's upstream gradient
// to the voxel that supplied the extremum.  Ties are broken by taking the
// first extremum in lexicographic (dz, dy, dx) order over the offsets of the
// element that fall inside the volume (a later offset wins only when it is
// strictly better).  Inputs holding NaN have no defined subgradient.
//
// Box element (separable).  Over a box clipped to the volume the offsets
// form a product set, and the lexicographically first extremum factorises
// exactly into three 1D first-extremum stages applied innermost first: at
// every voxel s the row stage picks dx among s + dx e_x, at every voxel q
// the plane stage picks dy among the row extrema at q + dy e_y, and at every
// output p the volume stage picks dz among the plane extrema at p + dz e_z.
// Each stage keeps the earliest offset among equal values, so the composed
// pick is the smallest (dz, dy, dx) among the maxima.  Erosion maximises the
// negated values (exact in f32).  Two z-streaming kernels:
//   argext_box: code[v] = xsel(v) | ysel(v) << 5 | zsel(v) << 10 (each field
//               offset + radius) -- the three stages' picks at voxel v;
//   gather_box: the adjoint of the composition, stage by stage in reverse
//               order: G1 = Z^T g (pushed into a ring of z accumulators),
//               G2 = Y^T G1, grad_in = X^T G2.  Every sum runs in a fixed
//               order (G1 by source slice, G2 by dy, grad_in by dx), so the
//               result does not depend on the tiling or the batching.
//
// Ball element (brute force over the element's offsets):
//   argext: code[p] = index of the chosen offset in the element's bounding
//           box, (dz + rz) (2ry + 1) (2rx + 1) + (dy + ry) (2rx + 1) + dx + rx;
//   gather: gin[j] = sum over offsets o of the element, in lexicographic
//           order, of g[j - o] where code[j - o] names o.
// Both stage a halo-padded 3D tile in LDS.  The gathers are deterministic
// sums (no atomics).
//
// sigma-gradient: per-block FP32 partials (from the fused Gaussian's dot
// epilogue, or from dot_partials_kernel) are reduced in FP64 in a fixed
// order by reduce_partials_f64.
#include <cmath>

#include "common.h"
#include "batch.h"
#include "tune.h"

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
__device__ __forceinline__ void argext_tile(const ChunkArgs &a, uint16_t *code, float *val, int op, int se, int rz,
                                            int ry, int rx, int bx, int by, int bz, float *sv)
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
        const int64_t o = (gz - a.out_o[0]) * a.out_sz + (gy - a.out_o[1]) * a.out_sy + (gx - a.out_o[2]);
        code[o] = (uint16_t)best_code;
        if (val) val[o] = best;  // the erosion / dilation itself
    }
}

template <typename T>
__global__ __launch_bounds__(kGT) void argext_kernel(ChunkArgs a, uint16_t *code, int op, int se, int rz, int ry,
                                                     int rx, int tiles_x, int tiles_y)
{
    extern __shared__ float sv[];
    int bx, by, bz;
    block_tile(tiles_x, tiles_y, bx, by, bz);
    argext_tile<T>(a, code, nullptr, op, se, rz, ry, rx, bx, by, bz, sv);
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
        argext_tile<T>(a, static_cast<uint16_t *>(const_cast<void *>(d.c[c].aux)), static_cast<float *>(d.c[c].out),
                       op, se, rz, ry, rx, bx, by, bz, sv);
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

// ------------------------------------------------------------ box, separable

constexpr int kSepThreads = 256;

__device__ __forceinline__ int wrap_slot(int s, int w) { return s < 0 ? s + w : (s >= w ? s - w : s); }

// LDS layout of argext_box: input slice (HY x SX), row extrema (HY x TX),
// ring of plane extrema (W x TY x TX) and their xy picks (u16), row picks (u8).
__host__ __device__ inline size_t argext_box_lds(int tx, int ty, int rz, int ry, int rx)
{
    const size_t hy = ty + 2 * ry, sx = tx + 2 * rx, w = 2 * rz + 1;
    return hy * sx * 4 + hy * tx * 4 + w * ty * tx * 6 + hy * tx;
}

// LDS layout of gather_box: ring of z accumulators (W x HY x SX), the
// y-adjoint slice (TY x SX) and the ring of codes (W x HY x SX, u16).
__host__ __device__ inline size_t gather_box_lds(int tx, int ty, int rz, int ry, int rx)
{
    const size_t hy = ty + 2 * ry, sx = tx + 2 * rx, w = 2 * rz + 1;
    return w * hy * sx * 6 + ty * sx * 4;
}

// Slice positions one thread stages per step (the halo'd column of a tile
// holds at most kSepThreads * kSepPF voxels; tiles are picked to fit).
constexpr int kSepPF = 8;

// Both separable kernels take the radii and the column tile either as
// template constants (CR: isotropic radius, CTX x CTY: tile; the common
// case, so that index arithmetic and the offset loops fold and unroll) or,
// with -1, as run-time arguments.

// Work items: (crop, TX x TY column, z range of zlen outputs).  in = volume,
// aux = code volume (written).  The next slice's values are loaded into
// registers while the current one is filtered.
template <typename T, int CR, int CTX, int CTY>
__global__ __launch_bounds__(kSepThreads) void argext_box_kernel(BatchDesc d, int erode, int rz_, int ry_, int rx_,
                                                                 int tx_, int ty_)
{
    const int rz = CR >= 0 ? CR : rz_, ry = CR >= 0 ? CR : ry_, rx = CR >= 0 ? CR : rx_;
    const int TX = CTX > 0 ? CTX : tx_, TY = CTY > 0 ? CTY : ty_;
    extern __shared__ float lds[];
    const int SX = TX + 2 * rx, HY = TY + 2 * ry, W = 2 * rz + 1, P = TY * TX;
    float *sv = lds;
    float *rv = sv + HY * SX;
    float *pv = rv + HY * TX;
    uint16_t *pc = reinterpret_cast<uint16_t *>(pv + W * P);
    uint8_t *rs = reinterpret_cast<uint8_t *>(pc + W * P);
    const int tid = threadIdx.x;
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const BatchCrop &k = d.c[c];
        const T *in = static_cast<const T *>(k.in);
        uint16_t *code = static_cast<uint16_t *>(const_cast<void *>(k.aux));
        float *vout = static_cast<float *>(k.out);  // the extremum itself, if wanted
        const int nz = k.n[0], ny = k.n[1], nx = k.n[2];
        const int64_t plane = (int64_t)ny * nx;
        const int x0 = bx * TX, y0 = by * TY;
        const int z_lo = bz * k.zlen, z_hi = min(nz, z_lo + k.zlen);
        // in-plane offsets of this thread's staged positions (clamped into
        // the volume; clamped positions are never picked)
        int32_t off[kSepPF];
#pragma unroll
        for (int j = 0; j < kSepPF; ++j) {
            const int e = tid + j * kSepThreads;
            const int ly = e / SX, lx = e - ly * SX;
            const int gy = min(max(y0 - ry + ly, 0), ny - 1), gx = min(max(x0 - rx + lx, 0), nx - 1);
            off[j] = gy * nx + gx;
        }
        T pf[kSepPF];
        auto fetch = [&](int t) __attribute__((always_inline)) {
            t = min(max(t, 0), nz - 1);
            const T *base = in + (int64_t)t * plane;
#pragma unroll
            for (int j = 0; j < kSepPF; ++j)
                if (tid + j * kSepThreads < HY * SX) pf[j] = base[off[j]];
        };
        const int t0 = z_lo - rz;
        fetch(t0);
        int slot = ((t0 % W) + W) % W;  // ring slot of slice t
        for (int t = t0; t < z_hi + rz; ++t) {
            const bool has_in = t >= 0 && t < nz;
            if (has_in) {
#pragma unroll
                for (int j = 0; j < kSepPF; ++j)
                    if (tid + j * kSepThreads < HY * SX) {
                        const float v = to_f32(pf[j]);
                        sv[tid + j * kSepThreads] = erode ? -v : v;
                    }
            }
            fetch(t + 1);
            lds_barrier();
            if (has_in) {
                // row stage at every row of the halo'd column
#pragma unroll
                for (int e = tid; e < HY * TX; e += kSepThreads) {
                    const int ly = e / TX, x = e - ly * TX, gx = x0 + x, gy = y0 - ry + ly;
                    if (gx >= nx || gy < 0 || gy >= ny) continue;
                    const int lo = max(-rx, -gx), hi = min(rx, nx - 1 - gx);
                    const float *row = sv + ly * SX + x + rx;
                    float best = row[lo];
                    int bi = lo;
#pragma unroll
                    for (int dx = -rx + 1; dx <= rx; ++dx) {
                        const float v = row[dx];
                        if (dx > lo && dx <= hi && v > best) {
                            best = v;
                            bi = dx;
                        }
                    }
                    rv[e] = best;
                    rs[e] = (uint8_t)(bi + rx);
                }
            }
            lds_barrier();
            if (has_in) {
                // plane stage; each thread keeps its own positions of the ring
#pragma unroll
                for (int e = tid; e < P; e += kSepThreads) {
                    const int y = e / TX, x = e - y * TX, gy = y0 + y;
                    if (gy >= ny || x0 + x >= nx) continue;
                    const int lo = max(-ry, -gy), hi = min(ry, ny - 1 - gy);
                    const float *col = rv + (y + ry) * TX + x;
                    float best = col[lo * TX];
                    int bi = lo;
#pragma unroll
                    for (int dy = -ry + 1; dy <= ry; ++dy) {
                        const float v = col[dy * TX];
                        if (dy > lo && dy <= hi && v > best) {
                            best = v;
                            bi = dy;
                        }
                    }
                    pv[slot * P + e] = best;
                    pc[slot * P + e] = (uint16_t)(rs[(y + ry) * TX + x] | (bi + ry) << 5);
                }
            }
            const int zo = t - rz;
            if (zo >= z_lo) {
                // volume stage of output slice zo (reads only this thread's
                // ring positions: no barrier needed)
                const int so = wrap_slot(slot - rz, W);
                const int lo = max(-rz, -zo), hi = min(rz, nz - 1 - zo);
#pragma unroll
                for (int e = tid; e < P; e += kSepThreads) {
                    const int y = e / TX, x = e - y * TX, gy = y0 + y, gx = x0 + x;
                    if (gy >= ny || gx >= nx) continue;
                    const int s_lo = wrap_slot(so + lo, W);
                    float best = pv[s_lo * P + e];
                    int bi = lo;
#pragma unroll
                    for (int dz = -rz + 1; dz <= rz; ++dz) {
                        const float v = pv[wrap_slot(so + dz, W) * P + e];
                        if (dz > lo && dz <= hi && v > best) {
                            best = v;
                            bi = dz;
                        }
                    }
                    code[(int64_t)zo * plane + (int64_t)gy * nx + gx] = (uint16_t)(pc[so * P + e] | (bi + rz) << 10);
                    if (vout) vout[(int64_t)zo * plane + (int64_t)gy * nx + gx] = erode ? -best : best;
                }
            }
            slot = slot + 1 == W ? 0 : slot + 1;
        }
        lds_barrier();
    }
}

// Work items as in argext_box.  in = upstream gradient g, aux = codes,
// out = grad_in.  The next slice's g and codes are loaded into registers
// while the current one is pushed and routed.
template <int CR, int CTX, int CTY>
__global__ __launch_bounds__(kSepThreads) void gather_box_kernel(BatchDesc d, int rz_, int ry_, int rx_, int tx_,
                                                                 int ty_)
{
    const int rz = CR >= 0 ? CR : rz_, ry = CR >= 0 ? CR : ry_, rx = CR >= 0 ? CR : rx_;
    const int TX = CTX > 0 ? CTX : tx_, TY = CTY > 0 ? CTY : ty_;
    extern __shared__ float lds[];
    const int SX = TX + 2 * rx, HY = TY + 2 * ry, W = 2 * rz + 1, H = HY * SX;
    float *acc = lds;
    float *g2 = acc + W * H;
    uint16_t *cr = reinterpret_cast<uint16_t *>(g2 + TY * SX);
    const int tid = threadIdx.x;
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const BatchCrop &k = d.c[c];
        const float *g = static_cast<const float *>(k.in);
        const uint16_t *code = static_cast<const uint16_t *>(k.aux);
        float *gin = static_cast<float *>(k.out);
        const int nz = k.n[0], ny = k.n[1], nx = k.n[2];
        const int64_t plane = (int64_t)ny * nx;
        const int x0 = bx * TX, y0 = by * TY;
        const int z_lo = bz * k.zlen, z_hi = min(nz, z_lo + k.zlen);
        // in-plane offsets of this thread's halo positions; -1 outside the
        // volume (no push, invalid code)
        int32_t off[kSepPF];
#pragma unroll
        for (int j = 0; j < kSepPF; ++j) {
            const int e = tid + j * kSepThreads;
            const int ly = e / SX, lx = e - ly * SX, gy = y0 - ry + ly, gx = x0 - rx + lx;
            off[j] = (e < H && gy >= 0 && gy < ny && gx >= 0 && gx < nx) ? gy * nx + gx : -1;
        }
        float pg[kSepPF];
        uint16_t pcd[kSepPF];
        auto fetch = [&](int t) __attribute__((always_inline)) {
            t = min(max(t, 0), nz - 1);
            const int64_t base = (int64_t)t * plane;
#pragma unroll
            for (int j = 0; j < kSepPF; ++j)
                if (off[j] >= 0) {
                    pg[j] = g[base + off[j]];
                    pcd[j] = code[base + off[j]];
                }
        };
        // the accumulator positions a thread clears are the ones it pushes to
        for (int e = tid; e < H; e += kSepThreads)
            for (int j = 0; j < W; ++j) acc[j * H + e] = 0.f;
        const int t0 = z_lo - rz;
        fetch(t0);
        int slot = ((t0 % W) + W) % W;
        for (int t = t0; t < z_hi + rz; ++t) {
            if (t >= 0 && t < nz) {
                // push slice t: G1[p + zsel(p)] += g[p] for outputs in range
#pragma unroll
                for (int j = 0; j < kSepPF; ++j) {
                    const int e = tid + j * kSepThreads;
                    if (e >= H) continue;
                    uint32_t cv = 0xffffu;
                    if (off[j] >= 0) {
                        cv = pcd[j];
                        const int dz = (int)(cv >> 10) - rz, q = t + dz;
                        if (q >= z_lo && q < z_hi) acc[wrap_slot(slot + dz, W) * H + e] += pg[j];
                    }
                    cr[slot * H + e] = (uint16_t)cv;
                }
            }
            fetch(t + 1);
            lds_barrier();
            const int qz = t - rz;
            const int sq = wrap_slot(slot - rz, W);
            if (qz >= z_lo) {
                // G2 = Y^T G1 over the x-halo'd rows of the tile
                const float *a = acc + sq * H;
                const uint16_t *cq = cr + sq * H;
#pragma unroll
                for (int e = tid; e < TY * SX; e += kSepThreads) {
                    const int y = e / SX, lx = e - y * SX;
                    float sum = 0.f;
#pragma unroll
                    for (int dy = -ry; dy <= ry; ++dy) {
                        const int q = (y + ry - dy) * SX + lx;
                        if (((cq[q] >> 5) & 31) == dy + ry) sum += a[q];
                    }
                    g2[e] = sum;
                }
            }
            lds_barrier();
            if (qz >= z_lo) {
                // grad_in = X^T G2, then release this slice's accumulators
                const uint16_t *cq = cr + sq * H;
#pragma unroll
                for (int e = tid; e < TY * TX; e += kSepThreads) {
                    const int y = e / TX, x = e - y * TX, gy = y0 + y, gx = x0 + x;
                    if (gy >= ny || gx >= nx) continue;
                    float sum = 0.f;
#pragma unroll
                    for (int dx = -rx; dx <= rx; ++dx) {
                        const int q = x + rx - dx;
                        if ((cq[(y + ry) * SX + q] & 31) == dx + rx) sum += g2[y * SX + q];
                    }
                    gin[(int64_t)qz * plane + (int64_t)gy * nx + gx] = sum;
                }
#pragma unroll
                for (int e = tid; e < H; e += kSepThreads) acc[sq * H + e] = 0.f;
            }
            slot = slot + 1 == W ? 0 : slot + 1;
        }
        lds_barrier();
    }
}

struct SepTile {
    int tx, ty;
};

// Largest column tile whose LDS fits 64 KiB (the kernels are written for
// any tile; wide tiles cut the halo re-reads).
inline bool sep_tile_fits(int tx, int ty, const int r[3])
{
    return (ty + 2 * r[1]) * (tx + 2 * r[2]) <= kSepThreads * kSepPF;
}

template <class F>
bool pick_sep_tile(F lds_of, const int r[3], SepTile &t, size_t &lds)
{
    static const SepTile cand[] = {{64, 8}, {64, 4}, {32, 4}, {32, 2}, {16, 2}, {16, 1}};
    for (const SepTile &c : cand) {
        const size_t b = lds_of(c.tx, c.ty);
        if (b <= 65536 && sep_tile_fits(c.tx, c.ty, r)) {
            t = c;
            lds = b;
            return true;
        }
    }
    return false;
}

// z-range length: whole-depth columns when there are enough of them to fill
// the device several times over, else shorter ranges (each range re-reads
// 2 rz halo slices).
inline int sep_zlen(const BatchDesc &d, int tx, int ty, int rz, int64_t capacity)
{
    int zlen = 256;
    const int floor_len = 8 * rz > 16 ? 8 * rz : 16;
    while (zlen > floor_len) {
        int64_t items = 0;
        for (int c = 0; c < d.n_crops; ++c)
            items += (int64_t)((d.c[c].n[2] + tx - 1) / tx) * ((d.c[c].n[1] + ty - 1) / ty) *
                     ((d.c[c].n[0] + zlen - 1) / zlen);
        if (items >= 4 * capacity) break;
        zlen /= 2;
    }
    return zlen;
}

inline int radius_code(const int r[3]) { return r[0] * 256 + r[1] * 16 + r[2]; }

// Tuned tile if recorded (and its LDS fits), else the widest fitting tile.
template <class F>
bool box_tile(int fam, uint64_t key, F lds_of, const int r[3], SepTile &tile, size_t &lds, int &zlen)
{
    Tile t;
    zlen = 0;
    if (tune_lookup(fam, key, t) && t.tx > 0 && t.ty > 0 && lds_of(t.tx, t.ty) <= 65536 &&
        sep_tile_fits(t.tx, t.ty, r)) {
        tile = SepTile{t.tx, t.ty};
        lds = lds_of(t.tx, t.ty);
        zlen = t.tz;
        return true;
    }
    return pick_sep_tile(lds_of, r, tile, lds);
}

// Specialised instance for isotropic radius r (1..4) on the 64 x 8 tile,
// else the run-time kernel.
constexpr int kSpecTX = 64, kSpecTY = 8;

template <typename T>
using ArgextFn = void (*)(BatchDesc, int, int, int, int, int, int);
using GatherFn = void (*)(BatchDesc, int, int, int, int, int);

template <typename T>
ArgextFn<T> argext_fn(const int r[3], const SepTile &t)
{
    if (r[0] == r[1] && r[1] == r[2] && t.tx == kSpecTX && t.ty == kSpecTY) {
        switch (r[0]) {
        case 1: return argext_box_kernel<T, 1, kSpecTX, kSpecTY>;
        case 2: return argext_box_kernel<T, 2, kSpecTX, kSpecTY>;
        case 3: return argext_box_kernel<T, 3, kSpecTX, kSpecTY>;
        case 4: return argext_box_kernel<T, 4, kSpecTX, kSpecTY>;
        default: break;
        }
    }
    return argext_box_kernel<T, -1, -1, -1>;
}

inline GatherFn gather_fn(const int r[3], const SepTile &t)
{
    if (r[0] == r[1] && r[1] == r[2] && t.tx == kSpecTX && t.ty == kSpecTY) {
        switch (r[0]) {
        case 1: return gather_box_kernel<1, kSpecTX, kSpecTY>;
        case 2: return gather_box_kernel<2, kSpecTX, kSpecTY>;
        case 3: return gather_box_kernel<3, kSpecTX, kSpecTY>;
        case 4: return gather_box_kernel<4, kSpecTX, kSpecTY>;
        default: break;
        }
    }
    return gather_box_kernel<-1, -1, -1>;
}

template <typename T>
bool argext_box_run(BatchDesc d, int op, const int r[3], hipStream_t s)
{
    SepTile tile;
    size_t lds;
    int zlen;
    if (!box_tile(TF_ARGEXT_BOX, tune_key_batch(TF_ARGEXT_BOX, radius_code(r), tune_type_code<T>(), d),
                  [&](int tx, int ty) { return argext_box_lds(tx, ty, r[0], r[1], r[2]); }, r, tile, lds, zlen))
        return false;
    const ArgextFn<T> fn = argext_fn<T>(r, tile);
    const int64_t cap = resident_blocks(fn, kSepThreads, lds);
    batch_layout(d, tile.tx, tile.ty, zlen > 0 ? zlen : sep_zlen(d, tile.tx, tile.ty, r[0], cap));
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap);
    if (grid > 0)
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kSepThreads), lds, s, d, op == HARPIA_ERODE ? 1 : 0, r[0],
                           r[1], r[2], tile.tx, tile.ty);
    return true;
}

bool gather_box_run(BatchDesc d, const int r[3], hipStream_t s)
{
    SepTile tile;
    size_t lds;
    int zlen;
    if (!box_tile(TF_GATHER_BOX, tune_key_batch(TF_GATHER_BOX, radius_code(r), 0, d),
                  [&](int tx, int ty) { return gather_box_lds(tx, ty, r[0], r[1], r[2]); }, r, tile, lds, zlen))
        return false;
    const GatherFn fn = gather_fn(r, tile);
    const int64_t cap = resident_blocks(fn, kSepThreads, lds);
    batch_layout(d, tile.tx, tile.ty, zlen > 0 ? zlen : sep_zlen(d, tile.tx, tile.ty, r[0], cap));
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap);
    if (grid > 0)
        hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kSepThreads), lds, s, d, r[0], r[1], r[2], tile.tx,
                           tile.ty);
    return true;
}

// One whole volume as a one-crop batch.
inline BatchDesc single_desc(const void *in, void *out, const void *aux, const int64_t n[3])
{
    BatchDesc d;
    d.n_crops = 1;
    d.c[0].in = in;
    d.c[0].out = out;
    d.c[0].aux = aux;
    for (int i = 0; i < 3; ++i) d.c[0].n[i] = (int32_t)n[i];
    return d;
}

// Brute-force LDS of the ball kernels (float values + u32 codes for the gather).
inline size_t ball_lds(const int r[3], size_t per_voxel)
{
    return per_voxel * (size_t)(kGZ + 2 * r[0]) * (kGY + 2 * r[1]) * (kGX + 2 * r[2]);
}

int64_t tiles_of(const ChunkArgs &a, int &tiles_x, int &tiles_y)
{
    tiles_x = (int)((a.out_e[2] + kGX - 1) / kGX);
    tiles_y = (int)((a.out_e[1] + kGY - 1) / kGY);
    return (int64_t)tiles_x * tiles_y * ((a.out_e[0] + kGZ - 1) / kGZ);
}

}  // namespace

constexpr int kMaxGradRadius = 8;

// Box: radii up to 8 per axis (the separable kernels' LDS fits for all of
// them).  Ball: the brute-force tile must fit 64 KiB of LDS, radius <= 4.
bool morph_grad_supported(int se, const int r[3])
{
    if (se == HARPIA_SE_BOX)
        return r[0] <= kMaxGradRadius && r[1] <= kMaxGradRadius && r[2] <= kMaxGradRadius;
    return ball_lds(r, 8) <= 65536;
}

static bool whole_volume(const ChunkArgs &a)
{
    for (int i = 0; i < 3; ++i)
        if (a.in_o[i] != 0 || a.out_o[i] != 0 || a.out_e[i] != a.n[i] || a.n[i] > (1 << 24)) return false;
    if (a.n[1] * a.n[2] >= ((int64_t)1 << 31)) return false;  // in-plane offsets are 32-bit
    return a.in_sy == a.n[2] && a.out_sy == a.n[2] && a.in_sz == a.n[1] * a.n[2] && a.out_sz == a.n[1] * a.n[2];
}

bool launch_argext(const ChunkArgs &a, harpia_dtype t, int op, int se, const int r[3], uint16_t *code, hipStream_t s)
{
    if (!morph_grad_supported(se, r)) return false;
    if (se == HARPIA_SE_BOX) {
        if (!whole_volume(a)) return false;
        const BatchDesc d = single_desc(a.in, nullptr, code, a.n);
        switch (t) {
        case HARPIA_F32: return argext_box_run<float>(d, op, r, s);
        case HARPIA_U16: return argext_box_run<uint16_t>(d, op, r, s);
        case HARPIA_U8: return argext_box_run<uint8_t>(d, op, r, s);
        case HARPIA_F16: return argext_box_run<_Float16>(d, op, r, s);
        case HARPIA_BF16: return argext_box_run<bf16_t>(d, op, r, s);
        }
        return false;
    }
    int tx, ty;
    const int64_t blocks = tiles_of(a, tx, ty);
    if (blocks == 0) return true;
    const size_t lds = ball_lds(r, sizeof(float));
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
    if (!morph_grad_supported(se, r)) return false;
    if (se == HARPIA_SE_BOX) {
        if (!whole_volume(a)) return false;
        return gather_box_run(single_desc(a.in, a.out, code, a.n), r, s);
    }
    int tx, ty;
    const int64_t blocks = tiles_of(a, tx, ty);
    if (blocks == 0) return true;
    const size_t lds = ball_lds(r, 8);
    hipLaunchKernelGGL(gather_kernel, dim3((uint32_t)blocks), dim3(kGT), lds, s, a, code, se, r[0], r[1], r[2], tx,
                       ty);
    return true;
}

bool launch_argext_batched(const BatchDesc &d0, harpia_dtype t, int op, int se, const int r[3], hipStream_t s)
{
    if (!morph_grad_supported(se, r) || t != HARPIA_F32) return false;
    if (se == HARPIA_SE_BOX) return argext_box_run<float>(d0, op, r, s);
    BatchDesc d = d0;
    batch_layout(d, kGX, kGY, kGZ);
    const size_t lds = ball_lds(r, sizeof(float));
    const int64_t cap = resident_blocks(argext_batched_kernel<float>, kGT, lds);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < 8192 ? cap : 8192);
    if (grid > 0)
        hipLaunchKernelGGL((argext_batched_kernel<float>), dim3((uint32_t)grid), dim3(kGT), lds, s, d, op, se, r[0],
                           r[1], r[2]);
    return true;
}

bool launch_gather_batched(const BatchDesc &d0, int se, const int r[3], hipStream_t s)
{
    if (!morph_grad_supported(se, r)) return false;
    if (se == HARPIA_SE_BOX) return gather_box_run(d0, r, s);
    BatchDesc d = d0;
    batch_layout(d, kGX, kGY, kGZ);
    const size_t lds = ball_lds(r, 8);
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
