/*
 * harpia.h -- C ABI of libharpia, an MI355X (gfx950) library of chunked,
 * halo-padded 3D volumetric filters: Gaussian smoothing and grayscale /
 * binary erosion, dilation, opening and closing (Section III-C of the
 * paper lists these filters among the library's CUDA algorithms), run chunk
 * by chunk under a strict device-memory budget so that volumes larger than
 * the budget still run (Section III-D, chunked processing).
 *
 * Volumes
 *   A volume is a dense C-ordered array [nz][ny][nx] (x contiguous, z
 *   slowest; chunks split along z as in Section III-D).  shape[] and every
 *   other per-axis array are ordered {z, y, x}.
 *
 * Pointers and ownership (Section I contribution 2, Section IV-C: the
 * library controls all device memory and releases it when a task ends)
 *   - `in` / `out` may both be device pointers (resident path: the call is
 *     asynchronous on ex->stream, no host<->device traffic) or both host
 *     pointers (streamed path: the library copies halo-padded chunks to the
 *     device, filters them and copies the core back; the call returns when
 *     `out` is complete).  Pinned host memory is copied by DMA directly;
 *     pageable host memory goes through pinned bounce buffers.
 *   - The caller owns `in` and `out`.  The library keeps no pointer after a
 *     call returns and holds no device memory between calls: every device
 *     byte it allocates is freed before the call returns (device path: after
 *     synchronising ex->stream if it had to allocate).
 *   - `in` and `out` must not overlap (HARPIA_ERR_ALIAS).
 *
 * Errors
 *   Every function returns a harpia_status; on error the thread-local
 *   message from harpia_last_error() says why, `out` is unspecified, and no
 *   device memory stays allocated.  Arguments are validated before any
 *   device work.
 *
 * Boundary
 *   Every filter uses half-sample symmetric reflection at the volume faces
 *   (index -1 reads voxel 0, index n reads voxel n-1; repeated for radii
 *   larger than the volume).  For erosion and dilation by box and ball
 *   elements this equals ignoring offsets outside the volume.
 *
 * Determinism
 *   Results are bitwise identical across runs and across chunk plans.
 *
 * Thread safety: every function may be called from several host threads.
 */
#ifndef HARPIA_H
#define HARPIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum harpia_status {
    HARPIA_OK = 0,
    HARPIA_ERR_ARG = -1,         /* invalid shape, sigma, radius, pointer... */
    HARPIA_ERR_DTYPE = -2,       /* unsupported dtype or dtype pair */
    HARPIA_ERR_BUDGET = -3,      /* not even the smallest chunk fits */
    HARPIA_ERR_OOM = -4,         /* a device or pinned allocation failed */
    HARPIA_ERR_HIP = -5,         /* a HIP runtime call failed */
    HARPIA_ERR_ALIAS = -6,       /* in and out overlap */
    HARPIA_ERR_UNSUPPORTED = -7  /* valid request this build does not run */
} harpia_status;

typedef enum harpia_dtype {
    HARPIA_U8 = 0,
    HARPIA_U16 = 1,
    HARPIA_F32 = 2,
    HARPIA_F16 = 3,   /* IEEE binary16 */
    HARPIA_BF16 = 4   /* bfloat16 */
} harpia_dtype;

/* Structuring elements.  BOX: |dz| <= rz, |dy| <= ry, |dx| <= rx.
 * BALL: dz^2 + dy^2 + dx^2 <= r^2 (isotropic: radius[0..2] must be equal). */
typedef enum harpia_se { HARPIA_SE_BOX = 0, HARPIA_SE_BALL = 1 } harpia_se;

typedef enum harpia_border { HARPIA_BORDER_REFLECT = 0 } harpia_border;

typedef enum harpia_morph_op { HARPIA_ERODE = 0, HARPIA_DILATE = 1 } harpia_morph_op;

/* harpia_exec.flags */
#define HARPIA_F_BINARY 0x1u        /* morphology: binarise the input as v != 0
                                       (unless a threshold is given); output
                                       is uint8 {0, 1} */
#define HARPIA_F_FORCE_CHUNKED 0x2u /* device path: use the chunk engine even
                                       when the whole volume fits the budget */
#define HARPIA_F_SIGMA_SUM 0x4u     /* Gaussian backward: grad_sigma receives
                                       one double, the sum of the three axis
                                       terms (the gradient of an isotropic
                                       sigma), reduced on the device in FP64 */
#define HARPIA_F_REUSE_CODES 0x8u   /* batched morphology backward: take the
                                       extremum codes that
                                       harpia_morph3d_forward_batched left in
                                       the workspace instead of recomputing
                                       them from the forward input */

/* Optional per-call statistics (filled when harpia_exec.stats != NULL). */
typedef struct harpia_stats {
    int64_t n_chunks;          /* chunks executed */
    int64_t bytes_h2d;         /* host -> device bytes copied */
    int64_t bytes_d2h;         /* device -> host bytes copied */
    int64_t peak_device_bytes; /* library-owned device bytes at peak */
    int64_t budget_bytes;      /* budget the call ran under */
    double wall_ms;            /* host wall time of the call */
    double kernel_ms;          /* host volumes: sum over chunks of the time
                                  the filter kernels took (HIP events on the
                                  compute stream around each chunk); 0 on
                                  the device path */
} harpia_stats;

/* Execution options; a NULL harpia_exec* means all defaults. */
typedef struct harpia_exec {
    size_t device_budget_bytes; /* cap on library device memory; the
                                   budget is min(cap, budget_fraction x free
                                   device memory); 0 => no cap (the
                                   HARPIA_DEVICE_BUDGET environment variable,
                                   in bytes, is the default cap) */
    double budget_fraction;     /* fraction of free device memory reserved
                                   for chunks (Section III-D, step 1);
                                   0 => HARPIA_BUDGET_FRACTION from the
                                   environment, else
                                   HARPIA_DEFAULT_BUDGET_FRACTION */
    int64_t chunk[3];           /* core chunk extent {z, y, x}; {0, 0, 0} =>
                                   the planner picks the deepest z-slab that
                                   fits (Section III-D, step 2) */
    void *stream;               /* hipStream_t of device-pointer calls; NULL
                                   => the default (null) stream */
    uint32_t flags;             /* HARPIA_F_* */
    harpia_stats *stats;        /* optional output */
} harpia_exec;

#define HARPIA_DEFAULT_BUDGET_FRACTION 0.5

/* A chunk plan (Section III-D, steps 1 and 2). */
typedef struct harpia_plan {
    int64_t shape[3];      /* volume */
    int64_t core[3];       /* core chunk extent (last chunk per axis may be
                              smaller) */
    int64_t grid[3];       /* chunks per axis */
    int32_t halo[3];       /* halo per side per axis */
    int32_t n_buffers;     /* buffer sets in flight (copy/compute overlap) */
    int64_t n_chunks;      /* grid[0] * grid[1] * grid[2] */
    size_t device_bytes;   /* device bytes the plan allocates (<= budget) */
    size_t budget_bytes;   /* budget the plan was made for */
} harpia_plan;

/* Thread-local message of the last failing call on this thread ("" if the
 * last call succeeded).  Valid until the next call on the same thread. */
const char *harpia_last_error(void);

/* Library version string, e.g. "harpia 0.1.0 gfx950". */
const char *harpia_version(void);

/* Truncation radius of a Gaussian: (int)(truncate * sigma + 0.5).
 * Returns -1 if sigma <= 0 or truncate < 0. */
int32_t harpia_gauss_radius(double sigma, double truncate);

/* Plan the chunking of a volume of `shape` whose filter needs `halo` voxels
 * per side (Section III-D: query free memory, reserve a fixed fraction,
 * compute the largest chunk that fits with its padding).  in_t / out_t give
 * the bytes per voxel of the staged input and output chunks.  ex may be
 * NULL.  The budget is min(cap, fraction x free device memory); on a host
 * without a GPU an explicit cap (ex->device_budget_bytes) is used as is, so
 * plans can be made there.
 * Errors: HARPIA_ERR_ARG (shape <= 0, halo < 0, out == NULL),
 *         HARPIA_ERR_DTYPE, HARPIA_ERR_BUDGET (a 1-slice chunk with its halo
 *         does not fit), HARPIA_ERR_HIP (free-memory query failed). */
harpia_status harpia_chunk_plan(const int64_t shape[3], harpia_dtype in_t,
                                harpia_dtype out_t, const int32_t halo[3],
                                const harpia_exec *ex, harpia_plan *out);

/* Gaussian smoothing (Section III-C, filtering suite):
 *   out = G_sigma * in, separable, taps w_k = exp(-k^2 / (2 s^2)) / sum,
 *   k = -r..r with r = (int)(truncate * s + 0.5) per axis, taps generated in
 *   FP64 and rounded to FP32, FP32 accumulation, reflect boundary.
 * sigma[3] per axis {z, y, x}, each > 0; truncate >= 0 (3.0 is usual).
 * dtype pairs (in -> out): F32->F32, U16->F32, U8->F32, F16->F16, F16->F32,
 *   BF16->BF16, BF16->F32.  16-bit outputs are rounded to nearest even.
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP. */
harpia_status harpia_gaussian3d(const void *in, harpia_dtype in_t, void *out,
                                harpia_dtype out_t, const int64_t shape[3],
                                const double sigma[3], double truncate,
                                harpia_border border, const harpia_exec *ex);

/* Mean (box) filter (Section III-C, smoothing filters of the filtering
 * suite): out = the average of `in` over the (2r+1)-box around each voxel,
 * i.e. the separable convolution with taps 1 / (2 r + 1) per axis (FP64,
 * rounded to FP32), FP32 accumulation, reflect boundary.
 * radius[3] in [0, 64] per axis {z, y, x}; dtype pairs as for
 * harpia_gaussian3d.  Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP. */
harpia_status harpia_mean3d(const void *in, harpia_dtype in_t, void *out,
                            harpia_dtype out_t, const int64_t shape[3],
                            const int32_t radius[3], harpia_border border,
                            const harpia_exec *ex);

/* Unsharp masking (Section III-C, edge enhancement of the filtering suite):
 *   out = in + amount * (in - G_sigma in) = (1 + amount) in - amount G_sigma in
 * with G_sigma the Gaussian of harpia_gaussian3d (same taps and boundary).
 * The Gaussian radii must be equal and in [1, 12] (the combination is an
 * epilogue of the fused kernel), else UNSUPPORTED.  amount finite.
 * dtype pairs as for harpia_gaussian3d.
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP, UNSUPPORTED. */
harpia_status harpia_unsharp3d(const void *in, harpia_dtype in_t, void *out,
                               harpia_dtype out_t, const int64_t shape[3],
                               const double sigma[3], double truncate,
                               double amount, harpia_border border,
                               const harpia_exec *ex);

/* Hessian of the Gaussian-smoothed volume (Section III-C, texture feature
 * extraction): out holds 6 float32 volumes, one after the other, with the
 * components zz, zy, zx, yy, yx, xx.  Component ab is the separable
 * correlation with, per axis, the taps of the derivative order that axis
 * takes (0, 1 or 2) of the normalised sampled Gaussian w (radius as for
 * harpia_gaussian3d): order 1 (k / s^2) w_k, order 2 ((k^2 - s^2) / s^4) w_k,
 * computed in FP64 and rounded to FP32; reflect boundary.  in: any dtype of
 * harpia_gaussian3d's pairs with float32 output.  Each component is one
 * filter pass (host volumes stream six times).
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP, UNSUPPORTED. */
harpia_status harpia_hessian3d(const void *in, harpia_dtype in_t, float *out,
                               const int64_t shape[3], const double sigma[3],
                               double truncate, harpia_border border,
                               const harpia_exec *ex);

/* Local thresholds (Section III-C, threshold algorithms of the label
 * editing module): out[p] = 1 if in[p] > T[p] else 0 (uint8), with
 *   HARPIA_THRESHOLD_MEAN:     T = m - offset,
 *   HARPIA_THRESHOLD_GAUSSIAN: T = G_sigma(in) - offset (taps and radius
 *                              as for harpia_gaussian3d with `truncate`),
 *   HARPIA_THRESHOLD_NIBLACK:  T = m + k s,
 *   HARPIA_THRESHOLD_SAUVOLA:  T = m (1 + k (s / r_param - 1)),
 * m the mean and s = sqrt(mean(in^2) - m^2) the standard deviation over the
 * (2 radius + 1)^3 box, reflect boundary, FP32 arithmetic (a voxel within
 * FP32 rounding of its threshold may fall on either side).
 * radius: 1..12 for mean, 1..6 for Niblack and Sauvola (unused for the
 * Gaussian, whose radius comes from sigma: 1..12).  t: U8, U16 or F32.
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP, UNSUPPORTED. */
typedef enum {
    HARPIA_THRESHOLD_MEAN = 0,
    HARPIA_THRESHOLD_GAUSSIAN = 1,
    HARPIA_THRESHOLD_NIBLACK = 2,
    HARPIA_THRESHOLD_SAUVOLA = 3
} harpia_threshold_method;

harpia_status harpia_local_threshold3d(const void *in, harpia_dtype t,
                                       uint8_t *out, const int64_t shape[3],
                                       harpia_threshold_method method,
                                       int32_t radius, double sigma,
                                       double truncate, double k,
                                       double r_param, double offset,
                                       harpia_border border,
                                       const harpia_exec *ex);

/* Otsu's global threshold (Section III-C, threshold algorithms) of an
 * integer volume, one histogram bin per value (U8: 256 bins, U16: 65536):
 * k = the split (class 0: values <= k) maximising w0 w1 (m0 - m1)^2, the
 * class counts w and means m, evaluated in FP64 from exact integer sums;
 * the first maximum wins; k = -1 when the volume holds one value.
 * out (device, may be NULL) receives (in > k) as uint8; threshold (host or
 * device pointer, may be NULL) receives k.  Device-resident volumes only
 * (else UNSUPPORTED); synchronises ex->stream before returning.
 * Errors: ARG, DTYPE, ALIAS, OOM, HIP, UNSUPPORTED. */
harpia_status harpia_otsu3d(const void *in, harpia_dtype t, uint8_t *out,
                            const int64_t shape[3], int64_t *threshold,
                            const harpia_exec *ex);

/* Sobel / Prewitt edge enhancement (Section III-C, filtering suite):
 *   G_a = central difference [-1, 0, 1] (in[i+1] - in[i-1]) along axis a,
 *         smoothed by [1, 2, 1] (HARPIA_EDGE_SOBEL) or [1, 1, 1]
 *         (HARPIA_EDGE_PREWITT) along the two other axes (unnormalised);
 *   out = sqrt(G_z^2 + G_y^2 + G_x^2), reflect boundary, FP32 arithmetic.
 * dtype pairs as for harpia_gaussian3d.
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP, UNSUPPORTED. */
typedef enum { HARPIA_EDGE_SOBEL = 0, HARPIA_EDGE_PREWITT = 1 } harpia_edge;

harpia_status harpia_edge3d(const void *in, harpia_dtype in_t, void *out,
                            harpia_dtype out_t, const int64_t shape[3],
                            harpia_edge kind, harpia_border border,
                            const harpia_exec *ex);

/* Erosion (min over the structuring element placed at each voxel) and
 * dilation (max) (Section III-C, label editing module).
 * t: dtype of `in`.  Grayscale: out has dtype t, results are exact; min
 * and max follow the IEEE 754 totalOrder of the values (-0 < +0, a NaN
 * orders beyond the infinities on the side of its sign).
 * Binary: if `threshold` is not NaN the input is binarised as in > threshold
 * (strict; the comparison is exact in the input's type), else with
 * HARPIA_F_BINARY as in != 0; `out` is then uint8 {0, 1}.
 * radius[3] >= 0 per axis {z, y, x}; BALL needs equal radii.
 * Errors: ARG, DTYPE, ALIAS, BUDGET, OOM, HIP, UNSUPPORTED. */
harpia_status harpia_erode3d(const void *in, void *out, harpia_dtype t,
                             const int64_t shape[3], harpia_se se,
                             const int32_t radius[3], double threshold,
                             harpia_border border, const harpia_exec *ex);

harpia_status harpia_dilate3d(const void *in, void *out, harpia_dtype t,
                              const int64_t shape[3], harpia_se se,
                              const int32_t radius[3], double threshold,
                              harpia_border border, const harpia_exec *ex);

/* Erosion and dilation with one element from a single read of the input
 * (both outputs of the label-editing module's morphology; their difference
 * is the morphological gradient).  Same rules as harpia_erode3d; the two
 * outputs must not overlap each other or `in`. */
harpia_status harpia_erode_dilate3d(const void *in, void *out_erode,
                                    void *out_dilate, harpia_dtype t,
                                    const int64_t shape[3], harpia_se se,
                                    const int32_t radius[3], double threshold,
                                    harpia_border border,
                                    const harpia_exec *ex);

/* A chain of erosions / dilations with one element, e.g. opening =
 * {HARPIA_ERODE, HARPIA_DILATE} and closing = {HARPIA_DILATE, HARPIA_ERODE}
 * (Section III-C lists both).  Each step is computed over the whole volume
 * before the next (the halo is the sum of the radii); the binarisation
 * rules of harpia_erode3d apply to the first step.  1 <= n_ops <= 8. */
harpia_status harpia_morph3d(const void *in, void *out, harpia_dtype t,
                             const int64_t shape[3],
                             const harpia_morph_op *ops, int32_t n_ops,
                             harpia_se se, const int32_t radius[3],
                             double threshold, harpia_border border,
                             const harpia_exec *ex);

/* ------------------------------------------------------------------
 * Gradients (an extension beyond the paper: differentiable filters).
 * Both run on device-resident volumes (device pointers; otherwise
 * HARPIA_ERR_UNSUPPORTED), on ex->stream.  When they allocate scratch they
 * synchronise ex->stream before freeing it, so they return with the results
 * complete.
 * ------------------------------------------------------------------ */

/* Gradient of y = G_sigma x (harpia_gaussian3d) for an upstream gradient
 * grad_out = dL/dy (float32):
 *   grad_in = G^T grad_out.  Under the half-sample reflect boundary every 1D
 *     factor of G is a symmetric matrix, so this is the same Gaussian applied
 *     to grad_out.  May be NULL.  float32.
 *   grad_sigma[a] = sum_p grad_out[p] * (d/d sigma_a (G x))[p] with the
 *     radii held fixed (d w_k / d sigma = w_k (k^2 - sum_j w_j j^2) / sigma^3),
 *     a = z, y, x: three doubles.  With HARPIA_F_SIGMA_SUM in ex->flags it
 *     is one double, the sum of the three (the gradient of an isotropic
 *     sigma, used for all three axes).  FP32 products summed per workgroup,
 *     workgroup partials summed in FP64 in a fixed order (deterministic).
 *     May be NULL, a host pointer (filled before return) or a device pointer
 *     (written on ex->stream).
 * x (dtype x_t, as for harpia_gaussian3d) is needed only for grad_sigma.
 * radius[3]: the radii the forward used (resolve them once with
 * harpia_gauss_radius and keep them; they are not recomputed from sigma). */
harpia_status harpia_gaussian3d_backward(const void *x, harpia_dtype x_t,
                                         const void *grad_out, void *grad_in,
                                         const int64_t shape[3],
                                         const double sigma[3],
                                         const int32_t radius[3],
                                         double *grad_sigma,
                                         const harpia_exec *ex);

/* harpia_gaussian3d_backward without any device allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as harpia_gaussian3d_backward, restricted to the single-launch
 * kernels: equal radii in [1, 12] and slices of fewer than 2^31 voxels
 * (else HARPIA_ERR_UNSUPPORTED).  Its scratch -- the sigma-gradient's FP32
 * workgroup partials and the FP64 results bound for a host grad_sigma --
 * is a fixed 4 MiB device array of the library, one per GPU, held until
 * the process ends; a volume whose partials exceed it (about 3 x 2^20
 * floats: 3 per 64 x 16 column tile and z range) is rejected with
 * HARPIA_ERR_ARG.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (several host threads or streams) race and must be
 * serialised by the caller.  With a device grad_sigma (or none) the call is
 * asynchronous on ex->stream; a host grad_sigma is filled before return. */
harpia_status harpia_gaussian3d_backward_noalloc(const void *x, harpia_dtype x_t,
                                                 const void *grad_out, void *grad_in,
                                                 const int64_t shape[3],
                                                 const double sigma[3],
                                                 const int32_t radius[3],
                                                 double *grad_sigma,
                                                 const harpia_exec *ex);

/* Subgradient of erosion (op = HARPIA_ERODE) or dilation of `in` (dtype t,
 * grayscale): every output voxel p sends grad_out[p] to the input voxel that
 * supplied its extremum, the first in lexicographic (dz, dy, dx) order over
 * the element's offsets inside the volume (ties go to the earliest offset):
 *   grad_in[j] = sum of grad_out[p] over the outputs p that chose j,
 * summed in a fixed order (no atomics; deterministic).  grad_out and grad_in
 * are float32.  Box radii up to 8 per axis; ball radius up to 4. */
harpia_status harpia_morph3d_backward(const void *in, harpia_dtype t,
                                      const void *grad_out, void *grad_in,
                                      const int64_t shape[3],
                                      harpia_morph_op op, harpia_se se,
                                      const int32_t radius[3],
                                      const harpia_exec *ex);

/* ------------------------------------------------------------------
 * Batched crops (an extension beyond the paper: many uneven volumes, e.g.
 * training crops or the edge chunks of a volume, in one persistent launch).
 * Each launch takes up to 64 crops whose (crop, tile) work items are strided
 * over the resident workgroups; larger batches are split into launches of
 * 64.  The crop table is passed by value in the kernel arguments, so these
 * calls allocate nothing and may be captured in a HIP graph.  All volumes
 * are dense float32 [nz][ny][nx] in device memory; calls are asynchronous on
 * ex->stream.
 * ------------------------------------------------------------------ */

typedef struct harpia_crop {
    const void *in;    /* volume read (forward input, or x for the sigma-gradient) */
    void *out;         /* volume written */
    const void *aux;   /* third volume (see each call) */
    int64_t shape[3];  /* {nz, ny, nx}, each in [1, 2^24] */
} harpia_crop;

/* Device workspace the batched backward calls need for these crops: FP32
 * partials of the sigma-gradient and the u16 extremum codes of every crop. */
size_t harpia_batch_workspace_bytes(const harpia_crop *crops, int32_t n_crops);

/* Gaussian of every crop (in -> out); float32, equal radii 1..12. */
harpia_status harpia_gaussian3d_batched(const harpia_crop *crops, int32_t n_crops,
                                        harpia_dtype in_t, harpia_dtype out_t,
                                        const double sigma[3], double truncate,
                                        const harpia_exec *ex);

/* Grayscale erosion / dilation of every crop (in -> out); with aux set on
 * every crop, out receives the erosion and aux the dilation.  float32,
 * equal radii 1..4. */
harpia_status harpia_morph3d_batched(const harpia_crop *crops, int32_t n_crops,
                                     harpia_dtype t, harpia_morph_op op,
                                     harpia_se se, const int32_t radius[3],
                                     const harpia_exec *ex);

/* Gaussian gradients over a batch, radii held fixed (equal, 1..12):
 * per crop in = x, aux = grad_out, out = grad_in (NULL on every crop to
 * skip).  grad_sigma (device pointer, 3 doubles, or NULL) receives
 * d/d sigma_{z,y,x} summed over all crops (one sigma shared by the batch);
 * with HARPIA_F_SIGMA_SUM in ex->flags, one double: the sum of the three.
 * FP32 workgroup partials in `workspace`, reduced in FP64 in fixed order. */
harpia_status harpia_gaussian3d_backward_batched(const harpia_crop *crops,
                                                 int32_t n_crops,
                                                 const double sigma[3],
                                                 const int32_t radius[3],
                                                 double *grad_sigma,
                                                 void *workspace,
                                                 size_t workspace_bytes,
                                                 const harpia_exec *ex);

/* Erosion / dilation of every crop (in -> out, float32, as
 * harpia_morph3d_batched) from the same pass that records, per output voxel,
 * the code of the offset that supplied its extremum (the first in
 * lexicographic (dz, dy, dx) order, as harpia_morph3d_backward routes) into
 * `workspace` (harpia_batch_workspace_bytes of these crops).  A later
 * harpia_morph3d_backward_batched on the same crops, element and workspace
 * with HARPIA_F_REUSE_CODES takes them instead of recomputing them, so the
 * forward input need not be kept.  Box radii up to 8, ball radius up to 4. */
harpia_status harpia_morph3d_forward_batched(const harpia_crop *crops,
                                             int32_t n_crops,
                                             harpia_morph_op op, harpia_se se,
                                             const int32_t radius[3],
                                             void *workspace,
                                             size_t workspace_bytes,
                                             const harpia_exec *ex);

/* Erosion / dilation subgradient over a batch: per crop in = forward input,
 * aux = grad_out, out = grad_in; rules of harpia_morph3d_backward.  The
 * codes live in `workspace` (harpia_batch_workspace_bytes); with
 * HARPIA_F_REUSE_CODES they are taken from a preceding
 * harpia_morph3d_forward_batched and `in` may be NULL. */
harpia_status harpia_morph3d_backward_batched(const harpia_crop *crops,
                                              int32_t n_crops,
                                              harpia_morph_op op, harpia_se se,
                                              const int32_t radius[3],
                                              void *workspace,
                                              size_t workspace_bytes,
                                              const harpia_exec *ex);

/* ------------------------------------------------------------------
 * Autotuner (an extension beyond the paper).  Each call below runs the
 * named operation on the caller's own operands once per tile candidate of
 * the kernels it launches (z-range split of the resident kernels; slices
 * per work item and column tile of the batched kernels), times the
 * candidates with HIP events on ex->stream (one warm-up, then `reps` timed
 * runs each; 0 -> 3), and records the fastest per (kernel, radius, element
 * type, extents or crop list).  Every later call in this process with the
 * same workload launches the recorded tile; a candidate is kept only if it
 * beats the library's own heuristic by 2 %.  Outputs and scratch operands
 * are overwritten.  Synchronous: ex->stream is idle on return.  Not for use
 * under graph capture.
 * ------------------------------------------------------------------ */

typedef struct harpia_tune_entry {
    char kernel[24];       /* kernel family */
    int32_t tile[3];       /* chosen {tx, ty, tz}; zeros = the heuristic */
    int32_t candidates;    /* candidates timed */
    float ms_heuristic;    /* mean time of the call with the heuristic tile */
    float ms_best;         /* mean time with the chosen tile */
} harpia_tune_entry;

typedef struct harpia_tune_report {
    int32_t n;
    harpia_tune_entry e[8];
} harpia_tune_report;

/* Tunes the fused Gaussian of harpia_gaussian3d on these operands (device
 * pointers).  report may be NULL. */
harpia_status harpia_autotune_gaussian3d(const void *in, harpia_dtype in_t,
                                         void *out, harpia_dtype out_t,
                                         const int64_t shape[3],
                                         const double sigma[3],
                                         double truncate, int32_t reps,
                                         const harpia_exec *ex,
                                         harpia_tune_report *report);

/* Tunes the morphology kernel of harpia_erode_dilate3d (grayscale, or
 * binary when a threshold or HARPIA_F_BINARY is given). */
harpia_status harpia_autotune_erode_dilate3d(const void *in, void *out_erode,
                                             void *out_dilate, harpia_dtype t,
                                             const int64_t shape[3],
                                             harpia_se se,
                                             const int32_t radius[3],
                                             double threshold, int32_t reps,
                                             const harpia_exec *ex,
                                             harpia_tune_report *report);

/* Tunes the batched kernels of a Gaussian -> dilation pipeline with its
 * gradients: harpia_gaussian3d_batched, harpia_morph3d_batched (dilation),
 * harpia_morph3d_backward_batched and the sigma-gradient of
 * harpia_gaussian3d_backward_batched.  Per crop: in = the Gaussian's input,
 * out and aux = two scratch volumes of the crop's shape (overwritten).
 * gauss_radius: the radii held fixed (equal, 1..12); workspace as for the
 * batched backward calls. */
harpia_status harpia_autotune_gauss_dilate_batched(
    const harpia_crop *crops, int32_t n_crops, const double sigma[3],
    const int32_t gauss_radius[3], harpia_se se, const int32_t morph_radius[3],
    void *workspace, size_t workspace_bytes, int32_t reps,
    const harpia_exec *ex, harpia_tune_report *report);

/* Recorded tiles: forget all, count, or save to / merge from a text file
 * ("harpia-tune 1" then one "key tx ty tz" line per workload). */
harpia_status harpia_tune_clear(void);
int64_t harpia_tune_entries(void);
harpia_status harpia_tune_save(const char *path);
harpia_status harpia_tune_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* HARPIA_H */
