// Gaussian smoothing kernels for gfx950 (templates; instantiated per dtype
// pair in gauss_<pair>.hip so the build compiles them in parallel) (the Gaussian filter of the
// library's filtering suite, Section III-C).
//
// out[z,y,x] = sum_{a,b,c} wz[a] wy[b] wx[c] in[R(z+a), R(y+b), R(x+c)]
// with half-sample reflection R and normalised sampled taps (FP64 -> FP32).
//
// Fused kernel (equal radius r on all axes, 1 <= r <= kGaussFusedMaxR):
//   one workgroup owns a TX x 16 tile of output columns (TX = 256 with 1024
//   threads for r <= 4, TX = 128 with 512 threads above; one 4-column quad
//   per thread) and streams along z over a range of output slices.  Per
//   input slice it
//     1. stages the (TX+2r) x (16+2r) patch in LDS (reflection applied on
//        load, converted to f32) -- the global loads of the next slice are
//        issued before the current slice is filtered, so HBM latency hides
//        behind the LDS work;
//     2. y pass from LDS, register-blocked 4 (r < 5) or 8 rows per work item;
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
#pragma once

#include <cstdint>
#include <utility>

#include "common.h"
#include "gauss_grid.h"
#include "batch.h"
#include "tune.h"

namespace harpia {


namespace gauss_detail {


constexpr int kNT = 256;  // threads per workgroup
constexpr int kMY = 4;    // rows per y-pass work item (sigma-gradient, Hessian)

// Rows per y-pass work item of the fused Gaussian: 8 for r >= 5 (each item
// reads 8 + 2r patch values for 8 outputs instead of 4 + 2r for 4, and the
// larger blocks cut LDS reads per output at the cost of transient
// registers), 4 below.
constexpr int fused_my(int r) { return r >= 5 ? 8 : 4; }


static_assert(kTX / 4 * kTY == kNT, "x pass maps one 4-column quad per thread");

// Store 4 consecutive outputs: one 16-byte (f32) or 8-byte (16-bit) store
// when all 4 are inside the region and the address is aligned, else element
// by element.  The aligned stores are non-temporal: the kernel never reads
// its output, and streaming it past the caches leaves them to the input
// slices.
template <typename T>
__device__ __forceinline__ void store4(T *p, const float v[4], int nvalid)
{
    constexpr uintptr_t kAlignMask = sizeof(T) * 4 - 1;
    if (nvalid == 4 && (reinterpret_cast<uintptr_t>(p) & kAlignMask) == 0) {
        if constexpr (sizeof(T) == 4) {
            typedef float v4f __attribute__((ext_vector_type(4)));
            const v4f q = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(q, reinterpret_cast<v4f *>(p));
        } else {
            uint16_t hb[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                T t = from_f32<T>(v[c]);
                hb[c] = *reinterpret_cast<uint16_t *>(&t);
            }
            typedef uint32_t v2u __attribute__((ext_vector_type(2)));
            const v2u q = {(uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16)};
            __builtin_nontemporal_store(q, reinterpret_cast<v2u *>(p));
        }
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < nvalid) p[c] = from_f32<T>(v[c]);
    }
}

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }
constexpr int lcm_int(int a, int b) { return a / gcd_int(a, b) * b; }

// Slices of input in flight per thread beyond the one being filtered.  With
// the LDS-only barrier one slice already overlaps a whole step; deeper rings
// make the compiler wait for them early (its wait counts merge
// conservatively across the step's branches).
constexpr int gauss_prefetch_depth(int) { return 1; }

// Output policies of the fused tile.  put(off, in_off, nvalid, v) receives
// the 4 finished outputs of one thread at element offset `off` of the
// output region (a.out layout) and `in_off` of the same voxels in the input
// region; nvalid of them lie inside the region.
//
// StoreOut stores them; with UNSHARP (amount a) it stores (1 + a) x - a v,
// x the input at the same voxel (read back from the input, which holds
// every output voxel).  A template flag, so that plain smoothing compiles
// to the same code as without the epilogue.
template <typename Tin, typename Tout, bool UNSHARP = false>
struct StoreOut {
    Tout *base;
    const Tin *in;
    float amount;
    Tin x[4];  // UNSHARP: the input at the next output's voxels, loaded a step early
    // Issue the loads of the next output's input values (one step ahead, so
    // their latency hides behind a step of filtering).
    __device__ __forceinline__ void prefetch(int64_t in_off, int nvalid)
    {
        if constexpr (UNSHARP) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nvalid) x[c] = in[in_off + c];
        }
    }
    __device__ __forceinline__ void put(int64_t off, int64_t, int nvalid, const float v[4])
    {
        if (nvalid <= 0) return;
        if constexpr (UNSHARP) {
            float u[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float xv = c < nvalid ? to_f32(x[c]) : 0.f;
                u[c] = fmaf(1.f + amount, xv, -amount * v[c]);
            }
            store4(base + off, u, nvalid);
        } else {
            store4(base + off, v, nvalid);
        }
    }
};

// One tile of the fused Gaussian: output columns [x0, x0 + kTX) x
// [y0, y0 + kTY) of the output region, slices [zo0, zo0 + zlen).
// PAR: bit a set (z = 1, y = 2, x = 4) when the taps of axis a are odd,
// c_{-k} = -c_k and c_0 = 0, with w[k] = c_k for k >= 1 (a first-derivative
// correlation, v[i + k] weighted by c_k); even taps otherwise.
template <typename Tin, int R, int D, class Out, int PAR = 0, int TX = kTX>
__device__ __forceinline__ void gauss_tile(const ChunkArgs &a, const FusedTaps &taps, int zlen, int bx, int by,
                                           int bz, int rot, Out &out)
{
    constexpr int NT = TX / 4 * kTY;  // threads: one 4-column quad each
    constexpr int P = 2 * R + 1;
    constexpr int PW = TX + 2 * R;  // patch columns
    constexpr int PH = kTY + 2 * R;  // patch rows
    constexpr int PSZ = PW * PH;
    constexpr int NLD = (PSZ + NT - 1) / NT;
    constexpr int QP = (PW + 3) & ~3;  // y-pass output pitch, 16-byte rows
    constexpr int MY = fused_my(R);
    constexpr int NYI = PW * (kTY / MY);
    constexpr int NH = 4 + 2 * R;  // x-pass inputs per quad
    constexpr int NH4 = (NH + 3) / 4;
    constexpr int QSZ = kTY * QP + 4 * NH4;

    // Double-buffered: slice i is filtered in y from sP[i & 1] into
    // sQ[i & 1] while slice i - 1 is filtered in x from sQ[(i - 1) & 1], so
    // one barrier per slice separates the phases.
    __shared__ float sP[2 * PSZ];
    __shared__ __attribute__((aligned(16))) float sQ[2 * QSZ];

    const int tid = threadIdx.x;
    const int64_t xbeg = a.out_o[2], ybeg = a.out_o[1];
    const int64_t xend = xbeg + a.out_e[2], yend = ybeg + a.out_e[1];
    const int64_t x0 = xbeg + (int64_t)bx * TX;
    const int64_t y0 = ybeg + (int64_t)by * kTY;
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

    // In-plane source offsets of this thread's patch elements; the same for
    // every slice.  Coordinates past the output region are clamped (they
    // only feed outputs that are never stored), so every reflected index
    // stays inside the input region.
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
    const int nsteps = (int)(zo1 - zo0) + 2 * R;  // input slices of this range

    // Prefetch ring of D slices: slot j mod D holds slice j.  Slot indices
    // are compile-time constants (the step loop is unrolled lcm(P, D)
    // times) and every fetch is unconditional (past the last slice it
    // re-reads the last one, which is never used), so the ring needs no
    // register moves and its loads stay in flight until they are staged.
    Tin pf[D][NLD];
    auto fetch = [&](int j, Tin(&dst)[NLD]) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const int64_t zl = reflect_index(s0 + j, a.n[0]) - a.in_o[0];
        const Tin *base = in + zl * a.in_sz;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * NT < PSZ) dst[k] = base[off[k]];
    };
    auto stage = [&](int j, const Tin(&src)[NLD]) __attribute__((always_inline)) {
        float *dst = sP + (j & 1) * PSZ;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * NT < PSZ) dst[tid + k * NT] = to_f32(src[k]);
    };

    const int qrow = tid / (TX / 4);
    const int qcol = (tid % (TX / 4)) * 4;
    const int64_t gy_out = y0 + qrow;
    const int64_t gx_out = x0 + qcol;
    const int nvalid = (gy_out < yend) ? (int)min((int64_t)4, xend - gx_out) : 0;
    const int64_t col_off = (gy_out - ybeg) * a.out_sy + (gx_out - xbeg);
    // y-pass items are dealt to the threads rotated by rot whole waves: NYI
    // is rarely a multiple of the workgroup, and rotating which waves take
    // the extra items between neighbouring workgroups spreads that work over
    // the SIMDs of a CU instead of loading the same SIMD in every workgroup.
    const int ytid = (tid + rot * 64) & (NT - 1);
    const int64_t in_col_off = (gy_out - a.in_o[1]) * a.in_sy + (gx_out - a.in_o[2]);

    float acc[P][4];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[j][c] = 0.f;

    static_for<D>([&](auto DD) { fetch(decltype(DD)::value, pf[decltype(DD)::value]); });
    stage(0, pf[0]);
    fetch(D, pf[0]);
    lds_barrier();

    // Step i: x and z passes of slice i - 1, y pass of slice i, staging of
    // slice i + 1.  Steps run 0 .. nsteps; the slot of output o in the z
    // ring is (o - s0) mod P, and slice j feeds outputs j - R .. j + R.
    constexpr int U = lcm_int(P, D);
    for (int base = 0; base <= nsteps; base += U) {
        static_for<U>([&](auto UU) {
            constexpr int u = decltype(UU)::value;
            const int i = base + u;
            if (i > nsteps) return;

            if (i >= 1) {
                // x pass of slice i - 1: 4 adjacent outputs from its y-pass row
                const float *q = sQ + ((i - 1) & 1) * QSZ;
                float h[NH4 * 4];
                const float4 *q4 = reinterpret_cast<const float4 *>(q + qrow * QP + qcol);
#pragma unroll
                for (int j = 0; j < NH4; ++j) {
                    const float4 t4 = q4[j];
                    h[4 * j + 0] = t4.x;
                    h[4 * j + 1] = t4.y;
                    h[4 * j + 2] = t4.z;
                    h[4 * j + 3] = t4.w;
                }
                float t[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float sacc;
                    if constexpr (PAR & 4) {
                        sacc = 0.f;
#pragma unroll
                        for (int k = 1; k <= R; ++k) sacc = fmaf(wx[k], h[c + R + k] - h[c + R - k], sacc);
                    } else {
                        sacc = wx[0] * h[c + R];
#pragma unroll
                        for (int k = 1; k <= R; ++k) sacc = fmaf(wx[k], h[c + R - k] + h[c + R + k], sacc);
                    }
                    t[c] = sacc;
                }
                // z pass: slice j = i - 1 feeds output o = j + d with the tap
                // c_{j - o} = c_{-d} (w|d| for even taps)
                static_for<P>([&](auto DD) {
                    constexpr int d = decltype(DD)::value - R;
                    constexpr int sl = (u - 1 + d + 2 * P) % P;
                    const float wd = (PAR & 1) ? (d == 0 ? 0.f : (d < 0 ? wz[-d] : -wz[d])) : wz[d < 0 ? -d : d];
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[sl][c] = (d == R) ? wd * t[c] : fmaf(wd, t[c], acc[sl][c]);
                });
            }
            if (i < nsteps) {
                // y pass of slice i: sP (PH x PW) -> sQ (kTY x PW)
                const float *p = sP + (i & 1) * PSZ;
                float *q = sQ + (i & 1) * QSZ;
#pragma unroll
                for (int itk = 0; itk < (NYI + NT - 1) / NT; ++itk) {
                    const int it = ytid + itk * NT;
                    if (itk == (NYI + NT - 1) / NT - 1 && it >= NYI) continue;
                    const int col = it % PW, rg = it / PW;
                    float v[MY + 2 * R];
#pragma unroll
                    for (int j = 0; j < MY + 2 * R; ++j) v[j] = p[(rg * MY + j) * PW + col];
#pragma unroll
                    for (int m = 0; m < MY; ++m) {
                        float sacc;
                        if constexpr (PAR & 2) {
                            sacc = 0.f;
#pragma unroll
                            for (int k = 1; k <= R; ++k) sacc = fmaf(wy[k], v[m + R + k] - v[m + R - k], sacc);
                        } else {
                            sacc = wy[0] * v[m + R];
#pragma unroll
                            for (int k = 1; k <= R; ++k) sacc = fmaf(wy[k], v[m + R - k] + v[m + R + k], sacc);
                        }
                        q[(rg * MY + m) * QP + col] = sacc;
                    }
                }
                // stage slice i + 1 and refill its slot with slice i + 1 + D
                constexpr int slot = (u + 1) % D;
                stage(i + 1, pf[slot]);
                fetch(i + 1 + D, pf[slot]);
            }
            // Output i - 1 - R is complete.  Stored after the fetch so that
            // staging the next slice does not wait for these stores (global
            // loads and stores share one in-order completion counter).  Its
            // ring slot is first rewritten by the next step.
            if (i >= 1 && i - 1 >= 2 * R) {
                constexpr int sl = (u - 1 - R + 2 * P) % P;
                const int64_t o = s0 + (i - 1) - R;
                out.put(col_off + (o - a.out_o[0]) * a.out_sz, in_col_off + (o - a.in_o[0]) * a.in_sz, nvalid,
                        acc[sl]);
            }
            // the output stored at step i + 1 (o = s0 + i - R) needs its
            // input voxels (unsharp epilogue): load them now
            if (i - R >= R && i < nsteps) {
                const int64_t o = s0 + i - R;
                out.prefetch(in_col_off + (o - a.in_o[0]) * a.in_sz, nvalid);
            }
            if (i < nsteps) lds_barrier();
        });
    }
}

// Sum of 256 values in a fixed order (wave butterflies, then the 4 wave
// sums); the result is valid in thread 0.
__device__ __forceinline__ float block_sum_256(float v)
{
    __shared__ float wsum[kNT / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    lds_barrier();
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    lds_barrier();
    return (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// All three sigma-gradient terms of one tile in one pass.  With G the
// Gaussian and D its sigma-derivative taps, every 1D factor is a symmetric
// matrix under the reflect boundary, so
//   S_z = <g, D_z G_y G_x x> = sum_s (G_y G_x x)[s] (D_z g)[s],
//   S_y = <g, G_z D_y G_x x> = sum_s (D_y G_x x)[s] (G_z g)[s],
//   S_x = <g, G_z G_y D_x x> = sum_s (G_y D_x x)[s] (G_z g)[s],
// sums over every voxel s.  The tile streams slices s of x through the y and
// x passes (both tap sets; no z halo of x is needed) while a ring of 2r+1
// slices of g (reflected in z) gives (G_z g)[s] and (D_z g)[s] in registers.
// x and g are dense [nz][ny][nx] volumes; g is float.  Adds this thread's
// share of S_z, S_y, S_x over slices [zo0, zo1) of the tile to sum[3].
template <typename Tin, int R, int D>
__device__ __forceinline__ void sigma3_tile(const Tin *x, const float *g, const int64_t n[3], const FusedTaps &wt,
                                            const FusedTaps &dt, int64_t x0, int64_t y0, int64_t zo0, int64_t zo1,
                                            float sum[3])
{
    constexpr int P = 2 * R + 1;
    constexpr int PW = kTX + 2 * R;
    constexpr int PH = kTY + 2 * R;
    constexpr int PSZ = PW * PH;
    constexpr int NLD = (PSZ + kNT - 1) / kNT;
    constexpr int QP = (PW + 3) & ~3;
    constexpr int NYI = PW * (kTY / kMY);
    constexpr int NH = 4 + 2 * R;
    constexpr int NH4 = (NH + 3) / 4;
    constexpr int QSZ = kTY * QP + 4 * NH4;

    __shared__ float sP[2 * PSZ];
    __shared__ __attribute__((aligned(16))) float sQG[2 * QSZ];  // y pass with G taps
    __shared__ __attribute__((aligned(16))) float sQD[2 * QSZ];  // y pass with D taps

    const int tid = threadIdx.x;
    const int64_t nz = n[0], ny = n[1], nx = n[2];
    const int64_t sy = nx, sz = nx * ny;
    if (zo0 >= zo1) return;

    float gz[R + 1], dz[R + 1], gy[R + 1], dy[R + 1], gx[R + 1], dx[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        gz[k] = wt.w[0][k];
        dz[k] = dt.w[0][k];
        gy[k] = wt.w[1][k];
        dy[k] = dt.w[1][k];
        gx[k] = wt.w[2][k];
        dx[k] = dt.w[2][k];
    }

    int32_t off[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
        const int e = tid + i * kNT;
        off[i] = 0;
        if (e < PSZ) {
            const int row = e / PW, col = e - (e / PW) * PW;
            int64_t yy = y0 - R + row;
            yy = yy > ny - 1 + R ? ny - 1 + R : yy;
            int64_t xx = x0 - R + col;
            xx = xx > nx - 1 + R ? nx - 1 + R : xx;
            off[i] = (int32_t)(reflect_index(yy, ny) * sy + reflect_index(xx, nx));
        }
    }

    const int nsteps = (int)(zo1 - zo0);  // slices of x this range filters
    Tin pf[D][NLD];
    auto fetch = [&](int j, Tin(&dst)[NLD]) __attribute__((always_inline)) {
        j = j < nsteps ? j : nsteps - 1;
        const Tin *base = x + (zo0 + j) * sz;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * kNT < PSZ) dst[k] = base[off[k]];
    };
    auto stage = [&](int j, const Tin(&src)[NLD]) __attribute__((always_inline)) {
        float *dst = sP + (j & 1) * PSZ;
#pragma unroll
        for (int k = 0; k < NLD; ++k)
            if (k < NLD - 1 || tid + k * kNT < PSZ) dst[tid + k * kNT] = to_f32(src[k]);
    };

    const int qrow = tid / (kTX / 4);
    const int qcol = (tid % (kTX / 4)) * 4;
    const int64_t y_out = y0 + qrow, x_out = x0 + qcol;
    const int nvalid = (y_out < ny) ? (int)min((int64_t)4, nx - x_out) : 0;
    const float *gcol = g + (nvalid > 0 ? y_out * sy + x_out : 0);

    // g ring: slot (z - (zo0 - R)) mod P holds g at the reflected slice z
    float gr[P][4];
    auto gload = [&](int64_t z, float(&dst)[4]) __attribute__((always_inline)) {
        const float *p = gcol + reflect_index(z, nz) * sz;
#pragma unroll
        for (int c = 0; c < 4; ++c) dst[c] = c < nvalid ? p[c] : 0.f;
    };
    static_for<2 * R>([&](auto K) { gload(zo0 - R + decltype(K)::value, gr[decltype(K)::value]); });

    static_for<D>([&](auto DD) { fetch(decltype(DD)::value, pf[decltype(DD)::value]); });
    stage(0, pf[0]);
    fetch(D, pf[0]);
    lds_barrier();

    // Step i: x pass and dot of slice s = zo0 + i - 1, y pass of slice
    // zo0 + i, staging of zo0 + i + 1, g of slice zo0 + i + R into the ring.
    constexpr int U = lcm_int(P, D);
    for (int base = 0; base <= nsteps; base += U) {
        static_for<U>([&](auto UU) {
            constexpr int u = decltype(UU)::value;
            const int i = base + u;
            if (i > nsteps) return;
            if (i >= 1) {
                const float *qg = sQG + ((i - 1) & 1) * QSZ + qrow * QP + qcol;
                const float *qd = sQD + ((i - 1) & 1) * QSZ + qrow * QP + qcol;
                float hg[NH4 * 4], hd[NH4 * 4];
#pragma unroll
                for (int j = 0; j < NH4; ++j) {
                    const float4 a4 = reinterpret_cast<const float4 *>(qg)[j];
                    const float4 b4 = reinterpret_cast<const float4 *>(qd)[j];
                    hg[4 * j] = a4.x, hg[4 * j + 1] = a4.y, hg[4 * j + 2] = a4.z, hg[4 * j + 3] = a4.w;
                    hd[4 * j] = b4.x, hd[4 * j + 1] = b4.y, hd[4 * j + 2] = b4.z, hd[4 * j + 3] = b4.w;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // in-plane values of slice s at column c
                    float tGG = gx[0] * hg[c + R], tGD = dx[0] * hg[c + R], tDG = gx[0] * hd[c + R];
#pragma unroll
                    for (int k = 1; k <= R; ++k) {
                        const float pg = hg[c + R - k] + hg[c + R + k];
                        tGG = fmaf(gx[k], pg, tGG);
                        tGD = fmaf(dx[k], pg, tGD);
                        tDG = fmaf(gx[k], hd[c + R - k] + hd[c + R + k], tDG);
                    }
                    // z-filtered g at slice s (ring slots of s - R .. s + R)
                    constexpr int sc = (u - 1 + R) % P;
                    float zg = gz[0] * gr[sc][c], zd = dz[0] * gr[sc][c];
                    static_for<R>([&](auto KK) {
                        constexpr int k = decltype(KK)::value + 1;
                        constexpr int sm = (u - 1 + R - k + P) % P, sp = (u - 1 + R + k) % P;
                        const float pr = gr[sm][c] + gr[sp][c];
                        zg = fmaf(gz[k], pr, zg);
                        zd = fmaf(dz[k], pr, zd);
                    });
                    sum[0] = fmaf(tGG, zd, sum[0]);
                    sum[1] = fmaf(tDG, zg, sum[1]);
                    sum[2] = fmaf(tGD, zg, sum[2]);
                }
            }
            // the ring slot of slice s - R is free now: load slice zo0 + i + R
            {
                constexpr int sl = (u + 2 * R) % P;
                gload(zo0 + i + R, gr[sl]);
            }
            if (i < nsteps) {
                const float *p = sP + (i & 1) * PSZ;
                float *q = sQG + (i & 1) * QSZ;
                float *qd = sQD + (i & 1) * QSZ;
#pragma unroll
                for (int itk = 0; itk < (NYI + kNT - 1) / kNT; ++itk) {
                    const int it = tid + itk * kNT;
                    if (itk == (NYI + kNT - 1) / kNT - 1 && it >= NYI) continue;
                    const int col = it % PW, rg = it / PW;
                    float v[kMY + 2 * R];
#pragma unroll
                    for (int j = 0; j < kMY + 2 * R; ++j) v[j] = p[(rg * kMY + j) * PW + col];
#pragma unroll
                    for (int m = 0; m < kMY; ++m) {
                        float sg = gy[0] * v[m + R], sd = dy[0] * v[m + R];
#pragma unroll
                        for (int k = 1; k <= R; ++k) {
                            const float pr = v[m + R - k] + v[m + R + k];
                            sg = fmaf(gy[k], pr, sg);
                            sd = fmaf(dy[k], pr, sd);
                        }
                        q[(rg * kMY + m) * QP + col] = sg;
                        qd[(rg * kMY + m) * QP + col] = sd;
                    }
                }
                constexpr int slot = (u + 1) % D;
                stage(i + 1, pf[slot]);
                fetch(i + 1 + D, pf[slot]);
                lds_barrier();
            }
        });
    }
}

// One workgroup per (tile, z range) of a dense volume; partials[b],
// partials[stride + b], partials[2 stride + b] get its S_z, S_y, S_x.
template <typename Tin, int R, int D = gauss_prefetch_depth(R)>
__global__ __launch_bounds__(kNT) void gauss_sigma3_kernel(const Tin *x, const float *g, int64_t nz, int64_t ny,
                                                           int64_t nx, FusedTaps wt, FusedTaps dt, int zlen,
                                                           int tiles_x, int tiles_y, float *partials, int64_t stride)
{
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = (int)(b % (uint32_t)tiles_x), by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
    const int bz = (int)(b / (uint32_t)(tiles_x * tiles_y));
    const int64_t n[3] = {nz, ny, nx};
    float sum[3] = {0.f, 0.f, 0.f};
    const int64_t z0 = (int64_t)bz * zlen;
    sigma3_tile<Tin, R, D>(x, g, n, wt, dt, (int64_t)bx * kTX, (int64_t)by * kTY, z0, min(z0 + zlen, nz), sum);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float t = block_sum_256(sum[a]);
        if (threadIdx.x == 0) partials[a * stride + b] = t;
    }
}

// Batched: persistent over the (crop, tile, z range) items; in = x, out =
// upstream gradient g.  One partial per workgroup and axis.
template <typename Tin, int R, int D = gauss_prefetch_depth(R)>
__global__ __launch_bounds__(kNT) void gauss_sigma3_batched_kernel(BatchDesc d, FusedTaps wt, FusedTaps dt,
                                                                   float *partials, int64_t stride)
{
    const int total = d.prefix[d.n_crops];
    float sum[3] = {0.f, 0.f, 0.f};
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const BatchCrop &k = d.c[c];
        const int64_t n[3] = {k.n[0], k.n[1], k.n[2]};
        const int64_t z0 = (int64_t)bz * k.zlen;
        sigma3_tile<Tin, R, D>(static_cast<const Tin *>(k.in), static_cast<const float *>(k.out), n, wt, dt,
                               (int64_t)bx * kTX, (int64_t)by * kTY, z0, min(z0 + (int64_t)k.zlen, n[0]), sum);
        lds_barrier();
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float t = block_sum_256(sum[a]);
        if (threadIdx.x == 0) partials[a * stride + blockIdx.x] = t;
    }
}

// Tile of logical block b (after xcd_remap, consecutive b run on one XCD at
// the same time).  SH = 0: row-major over (x, y, z ranges).  SH > 0: within
// each z range the tile rows are grouped into bands of SH rows, walked
// column by column, so the blocks one XCD holds at once cover a compact
// SH-row patch of tiles and share more of their y halos in that XCD's L2.
template <int SH = 0>
__device__ __forceinline__ void tile_of_block(uint32_t b, int tiles_x, int tiles_y, int &bx, int &by, int &bz)
{
    if constexpr (SH == 0) {
        bx = (int)(b % (uint32_t)tiles_x);
        by = (int)((b / (uint32_t)tiles_x) % (uint32_t)tiles_y);
        bz = (int)(b / (uint32_t)(tiles_x * tiles_y));
    } else {
        const uint32_t tiles = (uint32_t)(tiles_x * tiles_y);
        bz = (int)(b / tiles);
        const uint32_t rem = b % tiles;
        const uint32_t band = (uint32_t)SH * (uint32_t)tiles_x;
        const uint32_t sy = rem / band, idx = rem % band;
        const uint32_t hgt = min((uint32_t)SH, (uint32_t)tiles_y - sy * (uint32_t)SH);  // last band may be lower
        bx = (int)(idx / hgt);
        by = (int)(sy * (uint32_t)SH + idx % hgt);
    }
}

// Band height of the fused Gaussian's block order: 4 tile rows for r >= 5,
// whose 128 x 16 tiles stage 2r halo rows per 16 output rows (at r = 12 and
// 2048^3: 30.7 -> 28.9 ms); row-major below, where it measured slower.
constexpr int fused_band(int r) { return r >= 5 ? 4 : 0; }

template <typename Tin, typename Tout, int R, bool UNSHARP = false, int PAR = 0, int D = gauss_prefetch_depth(R)>
__global__ __launch_bounds__(fused_tx(R, UNSHARP) / 4 * kTY) void gauss_fused_kernel(ChunkArgs a, FusedTaps taps,
                                                                                   int zlen, int tiles_x,
                                                                                   int tiles_y)
{
    int bx, by, bz;
    const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
    tile_of_block<fused_band(R)>(b, tiles_x, tiles_y, bx, by, bz);
    StoreOut<Tin, Tout, UNSHARP> out{static_cast<Tout *>(a.out), static_cast<const Tin *>(a.in), taps.amount};
    gauss_tile<Tin, R, D, StoreOut<Tin, Tout, UNSHARP>, PAR, fused_tx(R, UNSHARP)>(a, taps, zlen, bx, by, bz,
                                                                                  (int)(b & 3u), out);
}

// Persistent batched Gaussian: workgroup b takes work items
// xcd_remap(b) + k * gridDim (so the workgroups of one XCD hold neighbouring
// tiles at any time); the LDS of the tile routine is reused between items.
template <typename Tin, typename Tout, int R, int D = gauss_prefetch_depth(R)>
__global__ __launch_bounds__(kNT) void gauss_batched_kernel(BatchDesc d, FusedTaps taps)
{
    const int total = d.prefix[d.n_crops];
    for (int w = (int)xcd_remap(blockIdx.x, gridDim.x); w < total; w += gridDim.x) {
        int c, bx, by, bz;
        batch_item(d, w, c, bx, by, bz);
        const ChunkArgs a = crop_args(d.c[c]);
        StoreOut<Tin, Tout> out{static_cast<Tout *>(a.out), static_cast<const Tin *>(a.in), taps.amount};
        gauss_tile<Tin, R, D>(a, taps, d.c[c].zlen, bx, by, bz, w & 3, out);
        lds_barrier();
    }
}

// One 1D pass along `axis` (0 z, 1 y, 2 x): dst = w * src, reflect along the
// axis.  src covers every reflected index; dst is dense or strided.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void gauss_pass_kernel(const Tin *src, int64_t s_sy, int64_t s_sz,
                                                         int64_t s_oz, int64_t s_oy, int64_t s_ox,
                                                         Tout *dst, int64_t d_sy, int64_t d_sz,
                                                         int64_t d_oz, int64_t d_oy, int64_t d_ox,
                                                         int64_t ez, int64_t ey, int64_t ex,
                                                         int axis, int64_t n_axis, GaussTaps taps)
{
    const int64_t total = ez * ey * ex;
    const int r = taps.r[axis];
    const bool odd = (taps.odd >> axis) & 1;  // c_{-k} = -c_k, c_0 = 0
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = id % ex, y = (id / ex) % ey, z = id / (ex * ey);
        const int64_t g[3] = {d_oz + z, d_oy + y, d_ox + x};
        float sacc = 0.f;
        for (int k = -r; k <= r; ++k) {
            int64_t c[3] = {g[0], g[1], g[2]};
            c[axis] = reflect_index(g[axis] + k, n_axis);
            const int64_t off = (c[0] - s_oz) * s_sz + (c[1] - s_oy) * s_sy + (c[2] - s_ox);
            float wk = taps.w[axis][k < 0 ? -k : k];
            if (odd) wk = k == 0 ? 0.f : (k < 0 ? -wk : wk);
            sacc = fmaf(wk, to_f32(src[off]), sacc);
        }
        dst[z * d_sz + y * d_sy + x] = from_f32<Tout>(sacc);
    }
}

template <typename Tin, typename Tout, int R, bool UNSHARP, int PAR = 0>
void launch_fused_u(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s)
{
    constexpr int TXF = fused_tx(R, UNSHARP);
    constexpr int NT = TXF / 4 * kTY;
    static const int64_t cap = resident_blocks(gauss_fused_kernel<Tin, Tout, R, UNSHARP, PAR>, NT);
    Tile t;
    // the tile width is part of the key: z splits tuned for other tiles do
    // not carry over
    const int code = tune_type_code<Tin>() * 8 + tune_type_code<Tout>() + (UNSHARP ? 64 : 0) + PAR * 128 +
                     TXF * 1024;
    const bool tuned = tune_lookup(TF_GAUSS, tune_key_volume(TF_GAUSS, R, code, a.out_e), t);
    const FusedGrid g = fused_grid(a, R, cap, tuned ? t.tz : 0, TXF);
    hipLaunchKernelGGL((gauss_fused_kernel<Tin, Tout, R, UNSHARP, PAR>), dim3((uint32_t)g.blocks), dim3(NT), 0, s,
                       a, fused_taps(taps), g.zlen, g.tiles_x, g.tiles_y);
}

// Three kernel families: plain smoothing (VAR 0), the unsharp epilogue
// (VAR 1) and odd derivative taps (VAR 2: the mixed Hessian components,
// built for float32 -> float32 only; other pairs take the unfused path).
// Each family has its own radius dispatch, so that one dtype pair's families
// can be compiled in separate units.
template <typename Tin, typename Tout, int R, int VAR>
bool launch_family(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s)
{
    if constexpr (VAR == 1) {
        launch_fused_u<Tin, Tout, R, true>(a, taps, s);
        return true;
    } else if constexpr (VAR == 2) {
        if constexpr (std::is_same<Tin, float>::value && std::is_same<Tout, float>::value) {
            switch (taps.odd) {
            case 3: launch_fused_u<Tin, Tout, R, false, 3>(a, taps, s); return true;
            case 5: launch_fused_u<Tin, Tout, R, false, 5>(a, taps, s); return true;
            case 6: launch_fused_u<Tin, Tout, R, false, 6>(a, taps, s); return true;
            default: return false;
            }
        }
        return false;
    } else {
        launch_fused_u<Tin, Tout, R, false, 0>(a, taps, s);
        return true;
    }
}

template <typename Tin, typename Tout, int VAR>
bool fused_family_run(int r, const ChunkArgs &a, const GaussTaps &taps, hipStream_t s)
{
    switch (r) {
#define HARPIA_CASE(RR) \
    case RR:            \
        return launch_family<Tin, Tout, RR, VAR>(a, taps, s);
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

template <typename Tin, typename Tout>
bool dispatch_fused(int r, const ChunkArgs &a, const GaussTaps &taps, hipStream_t s)
{
    if (taps.unsharp) return fused_family_run<Tin, Tout, 1>(r, a, taps, s);
    if (taps.odd) return fused_family_run<Tin, Tout, 2>(r, a, taps, s);
    return fused_family_run<Tin, Tout, 0>(r, a, taps, s);
}

template <typename Tin, typename Tout>
void launch_pass(const Tin *src, const Region &sr, Tout *dst, const Region &dr, int axis,
                 int64_t n_axis, const GaussTaps &taps, hipStream_t s)
{
    const int64_t total = dr.e[0] * dr.e[1] * dr.e[2];
    if (total == 0) return;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((gauss_pass_kernel<Tin, Tout>), dim3((uint32_t)blocks), dim3(256), 0, s, src, sr.sy,
                       sr.sz, sr.o[0], sr.o[1], sr.o[2], dst, dr.sy, dr.sz, dr.o[0], dr.o[1], dr.o[2],
                       dr.e[0], dr.e[1], dr.e[2], axis, n_axis, taps);
}

// Unfused: x pass over (input z, input y, output x) -> s1; y pass over
// (input z, output y, output x) -> s2; z pass -> out.
template <typename Tin, typename Tout>
void launch_unfused(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s, float *scratch)
{
    // Input region extent: every reflected index of the output region.
    // Reflected indices of [o - r, o + e + r) all lie in
    // [max(o - r, 0), min(o + e + r, n)).
    int64_t lo[3], hi[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int r = taps.r[ax];
        lo[ax] = a.out_o[ax] - r < 0 ? 0 : a.out_o[ax] - r;
        hi[ax] = a.out_o[ax] + a.out_e[ax] + r > a.n[ax] ? a.n[ax] : a.out_o[ax] + a.out_e[ax] + r;
    }
    Region src{const_cast<void *>(a.in), a.in_sy, a.in_sz, {a.in_o[0], a.in_o[1], a.in_o[2]}, {0, 0, 0}};
    Region r1{scratch, a.out_e[2], a.out_e[2] * (hi[1] - lo[1]), {lo[0], lo[1], a.out_o[2]},
              {hi[0] - lo[0], hi[1] - lo[1], a.out_e[2]}};
    float *s2p = scratch + r1.e[0] * r1.e[1] * r1.e[2];
    Region r2{s2p, a.out_e[2], a.out_e[2] * a.out_e[1], {lo[0], a.out_o[1], a.out_o[2]},
              {hi[0] - lo[0], a.out_e[1], a.out_e[2]}};
    Region dst{a.out, a.out_sy, a.out_sz, {a.out_o[0], a.out_o[1], a.out_o[2]},
               {a.out_e[0], a.out_e[1], a.out_e[2]}};
    launch_pass<Tin, float>(static_cast<const Tin *>(a.in), src, scratch, r1, 2, a.n[2], taps, s);
    launch_pass<float, float>(scratch, r1, s2p, r2, 1, a.n[1], taps, s);
    launch_pass<float, Tout>(s2p, r2, static_cast<Tout *>(a.out), dst, 0, a.n[0], taps, s);
}

template <typename Tin, typename Tout>
bool run(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s, void *scratch, size_t scratch_bytes)
{
    if (fused_ok(taps, a) && dispatch_fused<Tin, Tout>(taps.r[0], a, taps, s)) return true;
    if (taps.unsharp) return false;  // the unsharp epilogue lives in the fused kernel
    // the unfused passes, whatever the radii (odd taps of other dtype pairs,
    // slices too large for the fused kernel's 32-bit offsets)
    const int64_t need = (int64_t)gaussian_scratch_bytes(a.out_e, taps.r, false);
    if (scratch == nullptr || (int64_t)scratch_bytes < need) return false;
    launch_unfused<Tin, Tout>(a, taps, s, static_cast<float *>(scratch));
    return true;
}

// z range per batched work item: short enough that a batch of crops yields
// many items per resident workgroup, long enough to amortise the 2r warm-up.
constexpr int kBatchZ = 32;
constexpr int64_t kBatchMaxGrid = 8192;

template <typename Tin, typename Tout, int R>
void launch_batched(BatchDesc d, const GaussTaps &taps, hipStream_t s)
{
    static const int64_t cap = resident_blocks(gauss_batched_kernel<Tin, Tout, R>, kNT);
    Tile t;
    const bool tuned = tune_lookup(
        TF_GAUSS_BATCHED, tune_key_batch(TF_GAUSS_BATCHED, R, tune_type_code<Tin>() * 8 + tune_type_code<Tout>(), d), t);
    batch_layout(d, kTX, kTY, tuned && t.tz > 0 ? t.tz : kBatchZ);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < kBatchMaxGrid ? cap : kBatchMaxGrid);
    if (grid > 0)
        hipLaunchKernelGGL((gauss_batched_kernel<Tin, Tout, R>), dim3((uint32_t)grid), dim3(kNT), 0, s, d,
                           fused_taps(taps));
}

template <typename Tin, typename Tout>
bool dispatch_batched(int r, const BatchDesc &d, const GaussTaps &taps, hipStream_t s)
{
    switch (r) {
#define HARPIA_CASE(RR)                               \
    case RR:                                          \
        launch_batched<Tin, Tout, RR>(d, taps, s);    \
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

}  // namespace gauss_detail

template <typename Tin, typename Tout>
bool gauss_batched_run(const BatchDesc &d, const GaussTaps &taps, hipStream_t s)
{
    if (!(taps.r[0] == taps.r[1] && taps.r[1] == taps.r[2])) return false;
    return gauss_detail::dispatch_batched<Tin, Tout>(taps.r[0], d, taps, s);
}

namespace gauss_detail {

// z ranges of the three-term sigma-gradient: no z halo of x is read, so
// short ranges cost only the g ring's 2r-slice prologue; enough workgroups
// to fill the device several times, at most kMaxZRanges ranges.
inline int sigma3_zlen(int64_t nz, int64_t tiles, int64_t cap, int ranges)
{
    if (ranges <= 0) {
        ranges = 1;
        while (ranges < kMaxZRanges && tiles * ranges < 4 * cap && nz / (2 * ranges) >= 8) ranges *= 2;
    }
    if (ranges > kMaxZRanges) ranges = (int)kMaxZRanges;
    if (ranges > nz) ranges = (int)nz;
    return (int)((nz + ranges - 1) / ranges);
}

template <typename Tin, int R>
int64_t launch_sigma3(const Tin *x, const float *g, const int64_t n[3], const GaussTaps &wt, const GaussTaps &dt,
                      hipStream_t s, float *partials)
{
    static const int64_t cap = resident_blocks(gauss_sigma3_kernel<Tin, R>, kNT);
    const int tiles_x = (int)((n[2] + kTX - 1) / kTX), tiles_y = (int)((n[1] + kTY - 1) / kTY);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    Tile t;
    const bool tuned = tune_lookup(TF_GAUSS_DOT, tune_key_volume(TF_GAUSS_DOT, R, tune_type_code<Tin>() + 32, n), t);
    const int zlen = sigma3_zlen(n[0], tiles, cap, tuned ? t.tz : 0);
    const int64_t blocks = tiles * ((n[0] + zlen - 1) / zlen);
    hipLaunchKernelGGL((gauss_sigma3_kernel<Tin, R>), dim3((uint32_t)blocks), dim3(kNT), 0, s, x, g, n[0], n[1],
                       n[2], fused_taps(wt), fused_taps(dt), zlen, tiles_x, tiles_y, partials, blocks);
    return blocks;
}

template <typename Tin, int R>
int64_t launch_sigma3_batched(BatchDesc d, const GaussTaps &wt, const GaussTaps &dt, hipStream_t s, float *partials)
{
    static const int64_t cap = resident_blocks(gauss_sigma3_batched_kernel<Tin, R>, kNT);
    Tile t;
    const bool tuned = tune_lookup(TF_GAUSS_DOT_BATCHED,
                                   tune_key_batch(TF_GAUSS_DOT_BATCHED, R, tune_type_code<Tin>() + 32, d), t);
    batch_layout(d, kTX, kTY, tuned && t.tz > 0 ? t.tz : kBatchZ);
    const int64_t grid = batch_grid(d.prefix[d.n_crops], cap < kBatchMaxGrid ? cap : kBatchMaxGrid);
    if (grid > 0)
        hipLaunchKernelGGL((gauss_sigma3_batched_kernel<Tin, R>), dim3((uint32_t)grid), dim3(kNT), 0, s, d,
                           fused_taps(wt), fused_taps(dt), partials, grid);
    return grid;
}

}  // namespace gauss_detail

// Three-term sigma-gradient partials of a dense volume (x: Tin, g: float):
// returns the workgroup count nb (partials[a nb + b] for axis a), or -1.
template <typename Tin>
int64_t gauss_sigma3_run(const Tin *x, const float *g, const int64_t n[3], const GaussTaps &wt, const GaussTaps &dt,
                         hipStream_t s, float *partials)
{
    if (!(wt.r[0] == wt.r[1] && wt.r[1] == wt.r[2])) return -1;
    switch (wt.r[0]) {
#define HARPIA_CASE(RR) \
    case RR:            \
        return gauss_detail::launch_sigma3<Tin, RR>(x, g, n, wt, dt, s, partials);
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
        return -1;
    }
}

// Batched: per crop in = x, out = g; partials[a grid + b]; returns grid or -1.
template <typename Tin>
int64_t gauss_sigma3_batched_run(const BatchDesc &d, const GaussTaps &wt, const GaussTaps &dt, hipStream_t s,
                                 float *partials)
{
    if (!(wt.r[0] == wt.r[1] && wt.r[1] == wt.r[2])) return -1;
    switch (wt.r[0]) {
#define HARPIA_CASE(RR) \
    case RR:            \
        return gauss_detail::launch_sigma3_batched<Tin, RR>(d, wt, dt, s, partials);
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
        return -1;
    }
}

template <typename Tin, typename Tout>
bool gauss_run(const ChunkArgs &a, const GaussTaps &taps, hipStream_t s, void *scratch, size_t scratch_bytes)
{
    return gauss_detail::run<Tin, Tout>(a, taps, s, scratch, scratch_bytes);
}

}  // namespace harpia
