// Work lists of persistent batched launches: many uneven crops, each a dense
// [nz][ny][nx] volume in device memory, processed by one launch whose
// workgroups stride over the (crop, tile) work items.  The descriptor is a
// kernel argument (passed by value), so a batched launch needs no device
// allocation and can be captured in a HIP graph.
#pragma once

#include "common.h"

namespace harpia {

constexpr int kMaxBatch = 64;  // crops per launch; larger batches are split

struct BatchCrop {
    const void *in;   // volume read
    void *out;        // volume written (or the upstream gradient of a dot)
    const void *aux;  // third volume where a kernel needs one
    int32_t n[3];     // shape {z, y, x}
    int32_t tiles_x, tiles_y, zlen;
};

struct BatchDesc {
    int32_t n_crops;
    int32_t prefix[kMaxBatch + 1];  // work items before crop c
    BatchCrop c[kMaxBatch];
};

// The largest batched kernel argument list (the sigma-gradient: descriptor,
// two tap sets, partials pointer and stride) fits the 4 KiB kernel-argument
// space.
static_assert(sizeof(BatchDesc) + 2 * sizeof(FusedTaps) + 2 * sizeof(int64_t) <= 4096,
              "batch descriptor too large for the kernel arguments");

// Whole-volume chunk arguments of a crop (dense, origin 0).
__host__ __device__ inline ChunkArgs crop_args(const BatchCrop &c)
{
    ChunkArgs a;
    a.in = c.in;
    a.out = c.out;
    a.in_sy = a.out_sy = c.n[2];
    a.in_sz = a.out_sz = (int64_t)c.n[1] * c.n[2];
    for (int i = 0; i < 3; ++i) {
        a.in_o[i] = 0;
        a.out_o[i] = 0;
        a.out_e[i] = c.n[i];
        a.n[i] = c.n[i];
    }
    return a;
}

// Crop and tile of work item w.
__device__ __forceinline__ void batch_item(const BatchDesc &d, int w, int &c, int &bx, int &by, int &bz)
{
    c = 0;
    while (c + 1 < d.n_crops && d.prefix[c + 1] <= w) ++c;
    const int local = w - d.prefix[c];
    const int tx = d.c[c].tiles_x, ty = d.c[c].tiles_y;
    bx = local % tx;
    by = (local / tx) % ty;
    bz = local / (tx * ty);
}

// Fill tiles / z lengths / prefix for a batch with tiles of TX x TY columns
// and z ranges of `zlen` slices (clamped to each crop's depth).
inline void batch_layout(BatchDesc &d, int TX, int TY, int zlen)
{
    d.prefix[0] = 0;
    for (int c = 0; c < d.n_crops; ++c) {
        BatchCrop &k = d.c[c];
        k.tiles_x = (k.n[2] + TX - 1) / TX;
        k.tiles_y = (k.n[1] + TY - 1) / TY;
        k.zlen = zlen < k.n[0] ? zlen : k.n[0];
        const int zr = (k.n[0] + k.zlen - 1) / k.zlen;
        d.prefix[c + 1] = d.prefix[c] + k.tiles_x * k.tiles_y * zr;
    }
}

// Persistent grid: every resident workgroup, or fewer if there is less work.
inline int64_t batch_grid(int64_t items, int64_t capacity) { return items < capacity ? items : capacity; }

// Batched launches (see api.cpp for the C entry points).
bool launch_gauss_batched(const BatchDesc &d, harpia_dtype in_t, harpia_dtype out_t, const GaussTaps &taps,
                          hipStream_t s);
int64_t gauss_batched_max_partials();
// The three sigma-gradient terms over a batch in one pass (in = x, out =
// upstream gradient): partials[a grid + b]; returns grid, or -1.
int64_t launch_gauss_sigma3_batched(const BatchDesc &d, const GaussTaps &wt, const GaussTaps &dt, hipStream_t s,
                                    float *partials);
// Grayscale float32 erosion / dilation (isotropic radius 1..4) over a batch;
// with both = true, out = erosion and aux = dilation.
bool launch_morph_batched(const BatchDesc &d, harpia_dtype t, int op, int se, int r, bool both, hipStream_t s);
// Morphology subgradient over a batch: codes (aux = code volume, u16) then
// the gather (in = upstream gradient, aux = codes, out = grad_in).
bool launch_argext_batched(const BatchDesc &d, harpia_dtype t, int op, int se, const int r[3], hipStream_t s);
bool launch_gather_batched(const BatchDesc &d, int se, const int r[3], hipStream_t s);

}  // namespace harpia
