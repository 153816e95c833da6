// C ABI of libharpia (include/harpia.h): argument validation, error
// reporting and translation of each call into an engine job.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "engine.h"
#include "tune.h"

namespace harpia {

namespace {
thread_local std::string t_last_error;
}

void fail(harpia_status st, const std::string &msg) { throw Error{st, msg}; }

void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(HARPIA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

size_t dtype_size(harpia_dtype t)
{
    switch (t) {
    case HARPIA_U8: return 1;
    case HARPIA_U16: return 2;
    case HARPIA_F32: return 4;
    case HARPIA_F16: return 2;
    case HARPIA_BF16: return 2;
    }
    return 0;
}

const char *dtype_name(harpia_dtype t)
{
    switch (t) {
    case HARPIA_U8: return "u8";
    case HARPIA_U16: return "u16";
    case HARPIA_F32: return "f32";
    case HARPIA_F16: return "f16";
    case HARPIA_BF16: return "bf16";
    }
    return "?";
}

namespace {

template <class F>
harpia_status guarded(F &&f)
{
    try {
        f();
        t_last_error.clear();
        return HARPIA_OK;
    } catch (const Error &e) {
        t_last_error = e.message;
        return e.status;
    } catch (const std::bad_alloc &) {
        t_last_error = "host allocation failed";
        return HARPIA_ERR_OOM;
    } catch (const std::exception &e) {
        t_last_error = std::string("internal error: ") + e.what();
        return HARPIA_ERR_HIP;
    }
}

bool valid_dtype(int t) { return t >= HARPIA_U8 && t <= HARPIA_BF16; }

void check_shape(const int64_t *shape)
{
    if (!shape) fail(HARPIA_ERR_ARG, "shape is NULL");
    for (int a = 0; a < 3; ++a)
        if (shape[a] <= 0) fail(HARPIA_ERR_ARG, "shape extents must be > 0");
    const double total = (double)shape[0] * (double)shape[1] * (double)shape[2];
    if (total > 9.0e18) fail(HARPIA_ERR_ARG, "volume too large");
}

void check_exec(const harpia_exec *ex)
{
    if (!ex) return;
    if (ex->budget_fraction < 0.0 || ex->budget_fraction > 1.0)
        fail(HARPIA_ERR_ARG, "budget_fraction must be in [0, 1]");
    for (int a = 0; a < 3; ++a)
        if (ex->chunk[a] < 0) fail(HARPIA_ERR_ARG, "chunk extents must be >= 0");
}

void check_alias(const void *in, size_t in_bytes, const void *out, size_t out_bytes)
{
    const uintptr_t a0 = (uintptr_t)in, a1 = a0 + in_bytes;
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + out_bytes;
    if (a0 < b1 && b0 < a1) fail(HARPIA_ERR_ALIAS, "input and output overlap");
}

int64_t voxels(const int64_t *shape) { return shape[0] * shape[1] * shape[2]; }

bool gauss_pair_ok(harpia_dtype i, harpia_dtype o)
{
    return (i == HARPIA_F32 && o == HARPIA_F32) || (i == HARPIA_U16 && o == HARPIA_F32) ||
           (i == HARPIA_U8 && o == HARPIA_F32) || (i == HARPIA_F16 && (o == HARPIA_F16 || o == HARPIA_F32)) ||
           (i == HARPIA_BF16 && (o == HARPIA_BF16 || o == HARPIA_F32));
}

Stage gauss_stage(harpia_dtype in_t, harpia_dtype out_t, const double *sigma, double truncate)
{
    for (int a = 0; a < 3; ++a)
        if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) fail(HARPIA_ERR_ARG, "sigma must be finite and > 0");
    if (!(truncate >= 0.0) || !std::isfinite(truncate)) fail(HARPIA_ERR_ARG, "truncate must be finite and >= 0");
    Stage st;
    st.kind = Stage::GAUSS;
    st.in_t = in_t;
    st.out_t = out_t;
    int r[3];
    for (int a = 0; a < 3; ++a) {
        const double rr = truncate * sigma[a] + 0.5;
        if (rr >= (double)kMaxGaussRadius + 1.0)
            fail(HARPIA_ERR_UNSUPPORTED, "Gaussian radius above " + std::to_string(kMaxGaussRadius));
        r[a] = (int)rr;
        st.r[a] = r[a];
    }
    make_gauss_taps_r(sigma, r, st.taps);
    return st;
}

struct MorphArgs {
    harpia_se se;
    int r[3];
    bool binary;
    bool has_thr;
    double thr;
};

MorphArgs check_morph(harpia_dtype t, harpia_se se, const int32_t *radius, double threshold,
                      harpia_border border, const harpia_exec *ex)
{
    if (!valid_dtype(t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
    if (se != HARPIA_SE_BOX && se != HARPIA_SE_BALL) fail(HARPIA_ERR_ARG, "unknown structuring element");
    if (border != HARPIA_BORDER_REFLECT) fail(HARPIA_ERR_ARG, "only the reflect border is supported");
    if (!radius) fail(HARPIA_ERR_ARG, "radius is NULL");
    MorphArgs m;
    m.se = se;
    for (int a = 0; a < 3; ++a) {
        if (radius[a] < 0 || radius[a] > 64) fail(HARPIA_ERR_ARG, "radius must be in [0, 64]");
        m.r[a] = radius[a];
    }
    if (se == HARPIA_SE_BALL && (m.r[0] != m.r[1] || m.r[1] != m.r[2]))
        fail(HARPIA_ERR_ARG, "the ball element needs equal radii");
    m.has_thr = !std::isnan(threshold);
    m.thr = threshold;
    m.binary = m.has_thr || (ex && (ex->flags & HARPIA_F_BINARY));
    return m;
}

Stage morph_stage(harpia_dtype t, const MorphArgs &m, int op, bool first, Stage::Kind kind)
{
    Stage st;
    st.kind = kind;
    st.in_t = (first || !m.binary) ? t : HARPIA_U8;
    st.out_t = m.binary ? HARPIA_U8 : t;
    for (int a = 0; a < 3; ++a) st.r[a] = m.r[a];
    st.morph.op = op;
    st.morph.se = m.se;
    for (int a = 0; a < 3; ++a) st.morph.r[a] = m.r[a];
    st.morph.binary = m.binary;
    // Later steps of a binary chain read u8 {0, 1}: binarise as v != 0.
    st.morph.has_threshold = first && m.has_thr;
    st.morph.threshold = m.thr;
    return st;
}

}  // namespace
}  // namespace harpia

using namespace harpia;

extern "C" {

const char *harpia_last_error(void) { return t_last_error.c_str(); }

const char *harpia_version(void) { return "harpia 0.1.0 gfx950"; }

int32_t harpia_gauss_radius(double sigma, double truncate)
{
    if (!(sigma > 0.0) || !(truncate >= 0.0) || !std::isfinite(sigma) || !std::isfinite(truncate)) return -1;
    const double r = truncate * sigma + 0.5;
    if (r > 2.0e9) return -1;
    return (int32_t)r;
}

harpia_status harpia_chunk_plan(const int64_t shape[3], harpia_dtype in_t, harpia_dtype out_t,
                                const int32_t halo[3], const harpia_exec *ex, harpia_plan *out)
{
    return guarded([&] {
        check_shape(shape);
        check_exec(ex);
        if (!out) fail(HARPIA_ERR_ARG, "out is NULL");
        if (!halo) fail(HARPIA_ERR_ARG, "halo is NULL");
        if (!valid_dtype(in_t) || !valid_dtype(out_t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
        for (int a = 0; a < 3; ++a)
            if (halo[a] < 0) fail(HARPIA_ERR_ARG, "halo must be >= 0");
        // A single stencil step with the given halo, staged from the host.
        Stage st;
        std::memset(&st, 0, sizeof(st));
        st.kind = Stage::MORPH;
        st.in_t = in_t;
        st.out_t = out_t;
        for (int a = 0; a < 3; ++a) st.r[a] = halo[a];
        std::vector<Stage> stages{st};
        ChunkCost cost{true, dtype_size(in_t), dtype_size(out_t), 1, &stages};
        const size_t budget = resolve_budget(ex);
        const int64_t zero[3] = {0, 0, 0};
        plan_chunks(shape, halo, ex ? ex->chunk : zero, cost, budget, 3, *out);
    });
}

harpia_status harpia_gaussian3d(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                                const int64_t shape[3], const double sigma[3], double truncate,
                                harpia_border border, const harpia_exec *ex)
{
    return guarded([&] {
        if (!in || !out) fail(HARPIA_ERR_ARG, "in / out is NULL");
        check_shape(shape);
        check_exec(ex);
        if (!sigma) fail(HARPIA_ERR_ARG, "sigma is NULL");
        if (border != HARPIA_BORDER_REFLECT) fail(HARPIA_ERR_ARG, "only the reflect border is supported");
        if (!valid_dtype(in_t) || !valid_dtype(out_t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
        if (!gauss_pair_ok(in_t, out_t))
            fail(HARPIA_ERR_DTYPE, std::string("unsupported Gaussian dtype pair ") + dtype_name(in_t) + " -> " +
                                       dtype_name(out_t));
        const int64_t nv = voxels(shape);
        check_alias(in, nv * dtype_size(in_t), out, nv * dtype_size(out_t));
        Job job;
        job.in = in;
        job.out = out;
        job.out2 = nullptr;
        for (int a = 0; a < 3; ++a) job.n[a] = shape[a];
        job.stages.push_back(gauss_stage(in_t, out_t, sigma, truncate));
        job.ex = ex;
        run_job(job);
    });
}

// Shared checks of the Gaussian-family filters (one GAUSS stage).
static void run_gauss_family(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                             const int64_t shape[3], harpia_border border, const harpia_exec *ex, const Stage &st)
{
    if (!in || !out) fail(HARPIA_ERR_ARG, "in / out is NULL");
    check_shape(shape);
    check_exec(ex);
    if (border != HARPIA_BORDER_REFLECT) fail(HARPIA_ERR_ARG, "only the reflect border is supported");
    if (!valid_dtype(in_t) || !valid_dtype(out_t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
    if (!gauss_pair_ok(in_t, out_t))
        fail(HARPIA_ERR_DTYPE,
             std::string("unsupported dtype pair ") + dtype_name(in_t) + " -> " + dtype_name(out_t));
    const int64_t nv = voxels(shape);
    check_alias(in, nv * dtype_size(in_t), out, nv * dtype_size(out_t));
    Job job;
    job.in = in;
    job.out = out;
    job.out2 = nullptr;
    for (int a = 0; a < 3; ++a) job.n[a] = shape[a];
    job.stages.push_back(st);
    job.ex = ex;
    run_job(job);
}

harpia_status harpia_mean3d(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                            const int64_t shape[3], const int32_t radius[3], harpia_border border,
                            const harpia_exec *ex)
{
    return guarded([&] {
        if (!radius) fail(HARPIA_ERR_ARG, "radius is NULL");
        Stage st;
        std::memset(&st, 0, sizeof(st));
        st.kind = Stage::GAUSS;
        st.in_t = in_t;
        st.out_t = out_t;
        int r[3];
        for (int a = 0; a < 3; ++a) {
            if (radius[a] < 0 || radius[a] > kMaxGaussRadius)
                fail(HARPIA_ERR_ARG, "radius must be in [0, " + std::to_string(kMaxGaussRadius) + "]");
            r[a] = st.r[a] = radius[a];
        }
        make_mean_taps(r, st.taps);
        run_gauss_family(in, in_t, out, out_t, shape, border, ex, st);
    });
}

harpia_status harpia_otsu3d(const void *in, harpia_dtype t, uint8_t *out, const int64_t shape[3],
                            int64_t *threshold, const harpia_exec *ex)
{
    return guarded([&] {
        if (!in) fail(HARPIA_ERR_ARG, "in is NULL");
        check_shape(shape);
        check_exec(ex);
        if (t != HARPIA_U8 && t != HARPIA_U16) fail(HARPIA_ERR_DTYPE, "Otsu's threshold takes u8 or u16 volumes");
        if (t == HARPIA_U16 && (reinterpret_cast<uintptr_t>(in) & 1)) fail(HARPIA_ERR_ARG, "u16 volume not 2-byte aligned");
        const int64_t nv = voxels(shape);
        if (out) check_alias(in, nv * dtype_size(t), out, nv);
        if (!is_device_pointer(in) || (out && !is_device_pointer(out)))
            fail(HARPIA_ERR_UNSUPPORTED, "Otsu's threshold runs on device-resident volumes");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        DevBuf hist, res;
        const int nb = otsu_bins(t);
        hist.alloc((size_t)nb * sizeof(unsigned long long));
        res.alloc(sizeof(int64_t));
        check_hip(hipMemsetAsync(hist.p, 0, (size_t)nb * sizeof(unsigned long long), s), "hipMemsetAsync");
        if (!launch_otsu(in, t, nv, out, static_cast<unsigned long long *>(hist.p), static_cast<int64_t *>(res.p), s))
            fail(HARPIA_ERR_DTYPE, "no Otsu kernel for this dtype");
        check_hip(hipGetLastError(), "kernel launch");
        if (threshold)
            check_hip(hipMemcpyAsync(threshold, res.p, sizeof(int64_t), hipMemcpyDefault, s), "hipMemcpyAsync");
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    });
}

harpia_status harpia_local_threshold3d(const void *in, harpia_dtype t, uint8_t *out, const int64_t shape[3],
                                       harpia_threshold_method method, int32_t radius, double sigma, double truncate,
                                       double k, double r_param, double offset, harpia_border border,
                                       const harpia_exec *ex)
{
    return guarded([&] {
        if (!in || !out) fail(HARPIA_ERR_ARG, "in / out is NULL");
        check_shape(shape);
        check_exec(ex);
        if (border != HARPIA_BORDER_REFLECT) fail(HARPIA_ERR_ARG, "only the reflect border is supported");
        if (method < HARPIA_THRESHOLD_MEAN || method > HARPIA_THRESHOLD_SAUVOLA)
            fail(HARPIA_ERR_ARG, "unknown threshold method");
        if (t != HARPIA_U8 && t != HARPIA_U16 && t != HARPIA_F32)
            fail(HARPIA_ERR_DTYPE, "local thresholds take u8, u16 or f32 volumes");
        if (!std::isfinite(k) || !std::isfinite(offset) || !(r_param > 0.0) || !std::isfinite(r_param))
            fail(HARPIA_ERR_ARG, "k and offset must be finite, r_param finite and > 0");
        Stage st;
        std::memset(&st, 0, sizeof(st));
        st.kind = Stage::THRESH;
        st.in_t = t;
        st.out_t = HARPIA_U8;
        if (method == HARPIA_THRESHOLD_GAUSSIAN) {
            const double sg[3] = {sigma, sigma, sigma};
            const Stage g = gauss_stage(t == HARPIA_F32 ? HARPIA_F32 : HARPIA_U16, HARPIA_F32, sg, truncate);
            for (int a = 0; a < 3; ++a) st.r[a] = g.r[a];
            st.taps = g.taps;
        } else {
            int r[3] = {radius, radius, radius};
            make_mean_taps(r, st.taps);
            for (int a = 0; a < 3; ++a) st.r[a] = radius;
        }
        const int maxr = local_threshold_max_radius((int)method);
        if (st.r[0] < 1 || st.r[0] > maxr)
            fail(HARPIA_ERR_UNSUPPORTED, "threshold radius must be in [1, " + std::to_string(maxr) + "]");
        st.thr_method = (int)method;
        st.thr_k = (float)k;
        st.thr_r = (float)r_param;
        st.thr_offset = (float)offset;
        const int64_t nv = voxels(shape);
        check_alias(in, nv * dtype_size(t), out, nv);
        Job job;
        job.in = in;
        job.out = out;
        job.out2 = nullptr;
        for (int a = 0; a < 3; ++a) job.n[a] = shape[a];
        job.stages.push_back(st);
        job.ex = ex;
        run_job(job);
    });
}

harpia_status harpia_edge3d(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                            const int64_t shape[3], harpia_edge kind, harpia_border border, const harpia_exec *ex)
{
    return guarded([&] {
        if (kind != HARPIA_EDGE_SOBEL && kind != HARPIA_EDGE_PREWITT) fail(HARPIA_ERR_ARG, "unknown edge operator");
        Stage st;
        std::memset(&st, 0, sizeof(st));
        st.kind = Stage::EDGE;
        st.in_t = in_t;
        st.out_t = out_t;
        for (int a = 0; a < 3; ++a) st.r[a] = 1;
        st.edge = (int)kind;
        run_gauss_family(in, in_t, out, out_t, shape, border, ex, st);
    });
}

static Region whole_region(const void *p, const int64_t *n);

harpia_status harpia_hessian3d(const void *in, harpia_dtype in_t, float *out, const int64_t shape[3],
                               const double sigma[3], double truncate, harpia_border border, const harpia_exec *ex)
{
    return guarded([&] {
        if (!out) fail(HARPIA_ERR_ARG, "out is NULL");
        if (!sigma) fail(HARPIA_ERR_ARG, "sigma is NULL");
        check_shape(shape);
        const Stage base = gauss_stage(in_t, HARPIA_F32, sigma, truncate);
        const int64_t nv = voxels(shape);
        // device-resident float32 volumes with small equal radii: two passes
        // of three components (one read of the input each)
        if (in && in_t == HARPIA_F32 && border == HARPIA_BORDER_REFLECT &&
            !(ex && (ex->flags & HARPIA_F_FORCE_CHUNKED)) && is_device_pointer(in) && is_device_pointer(out)) {
            check_exec(ex);
            check_alias(in, nv * 4, out, 6 * nv * 4);
            hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
            const ChunkArgs a = make_chunk_args(whole_region(in, shape), whole_region(out, shape), shape);
            if (launch_hessian_fused(a, in_t, sigma, base.r, nv, s)) {
                check_hip(hipGetLastError(), "kernel launch");
                return;
            }
        }
        static const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        for (int c = 0; c < 6; ++c) {
            int order[3] = {0, 0, 0};
            ++order[pairs[c][0]];
            ++order[pairs[c][1]];
            Stage st = base;
            make_gauss_deriv_taps(sigma, base.r, order, st.taps);
            run_gauss_family(in, in_t, out + c * nv, HARPIA_F32, shape, border, ex, st);
        }
    });
}

harpia_status harpia_unsharp3d(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                               const int64_t shape[3], const double sigma[3], double truncate, double amount,
                               harpia_border border, const harpia_exec *ex)
{
    return guarded([&] {
        if (!sigma) fail(HARPIA_ERR_ARG, "sigma is NULL");
        if (!std::isfinite(amount)) fail(HARPIA_ERR_ARG, "amount must be finite");
        Stage st = gauss_stage(in_t, out_t, sigma, truncate);
        if (!(st.r[0] == st.r[1] && st.r[1] == st.r[2]) || st.r[0] < 1 || st.r[0] > kGaussFusedMaxR)
            fail(HARPIA_ERR_UNSUPPORTED, "unsharp masking needs equal Gaussian radii in [1, " +
                                             std::to_string(kGaussFusedMaxR) + "]");
        st.taps.amount = (float)amount;
        st.taps.unsharp = 1;
        run_gauss_family(in, in_t, out, out_t, shape, border, ex, st);
    });
}

static harpia_status morph_common(const void *in, void *out, harpia_dtype t, const int64_t shape[3],
                                  const harpia_morph_op *ops, int32_t n_ops, harpia_se se,
                                  const int32_t radius[3], double threshold, harpia_border border,
                                  const harpia_exec *ex)
{
    return guarded([&] {
        if (!in || !out) fail(HARPIA_ERR_ARG, "in / out is NULL");
        check_shape(shape);
        check_exec(ex);
        if (!ops || n_ops < 1 || n_ops > 8) fail(HARPIA_ERR_ARG, "n_ops must be in [1, 8]");
        for (int i = 0; i < n_ops; ++i)
            if (ops[i] != HARPIA_ERODE && ops[i] != HARPIA_DILATE) fail(HARPIA_ERR_ARG, "unknown morphology op");
        const MorphArgs m = check_morph(t, se, radius, threshold, border, ex);
        const int64_t nv = voxels(shape);
        const harpia_dtype out_t = m.binary ? HARPIA_U8 : t;
        check_alias(in, nv * dtype_size(t), out, nv * dtype_size(out_t));
        Job job;
        job.in = in;
        job.out = out;
        job.out2 = nullptr;
        for (int a = 0; a < 3; ++a) job.n[a] = shape[a];
        for (int i = 0; i < n_ops; ++i) job.stages.push_back(morph_stage(t, m, (int)ops[i], i == 0, Stage::MORPH));
        job.ex = ex;
        run_job(job);
    });
}

harpia_status harpia_erode3d(const void *in, void *out, harpia_dtype t, const int64_t shape[3], harpia_se se,
                             const int32_t radius[3], double threshold, harpia_border border,
                             const harpia_exec *ex)
{
    const harpia_morph_op op = HARPIA_ERODE;
    return morph_common(in, out, t, shape, &op, 1, se, radius, threshold, border, ex);
}

harpia_status harpia_dilate3d(const void *in, void *out, harpia_dtype t, const int64_t shape[3], harpia_se se,
                              const int32_t radius[3], double threshold, harpia_border border,
                              const harpia_exec *ex)
{
    const harpia_morph_op op = HARPIA_DILATE;
    return morph_common(in, out, t, shape, &op, 1, se, radius, threshold, border, ex);
}

harpia_status harpia_morph3d(const void *in, void *out, harpia_dtype t, const int64_t shape[3],
                             const harpia_morph_op *ops, int32_t n_ops, harpia_se se, const int32_t radius[3],
                             double threshold, harpia_border border, const harpia_exec *ex)
{
    return morph_common(in, out, t, shape, ops, n_ops, se, radius, threshold, border, ex);
}

harpia_status harpia_erode_dilate3d(const void *in, void *out_erode, void *out_dilate, harpia_dtype t,
                                    const int64_t shape[3], harpia_se se, const int32_t radius[3],
                                    double threshold, harpia_border border, const harpia_exec *ex)
{
    return guarded([&] {
        if (!in || !out_erode || !out_dilate) fail(HARPIA_ERR_ARG, "in / out is NULL");
        check_shape(shape);
        check_exec(ex);
        const MorphArgs m = check_morph(t, se, radius, threshold, border, ex);
        const int64_t nv = voxels(shape);
        const harpia_dtype out_t = m.binary ? HARPIA_U8 : t;
        check_alias(in, nv * dtype_size(t), out_erode, nv * dtype_size(out_t));
        check_alias(in, nv * dtype_size(t), out_dilate, nv * dtype_size(out_t));
        check_alias(out_erode, nv * dtype_size(out_t), out_dilate, nv * dtype_size(out_t));
        Job job;
        job.in = in;
        job.out = out_erode;
        job.out2 = out_dilate;
        for (int a = 0; a < 3; ++a) job.n[a] = shape[a];
        job.stages.push_back(morph_stage(t, m, HARPIA_ERODE, true, Stage::MORPH_BOTH));
        job.ex = ex;
        run_job(job);
    });
}


static Region whole_region(const void *p, const int64_t *n)
{
    Region r;
    r.ptr = const_cast<void *>(p);
    r.sy = n[2];
    r.sz = n[1] * n[2];
    for (int a = 0; a < 3; ++a) {
        r.o[a] = 0;
        r.e[a] = n[a];
    }
    return r;
}

harpia_status harpia_gaussian3d_backward(const void *x, harpia_dtype x_t, const void *grad_out, void *grad_in,
                                         const int64_t shape[3], const double sigma[3], const int32_t radius[3],
                                         double *grad_sigma, const harpia_exec *ex)
{
    return guarded([&] {
        check_shape(shape);
        check_exec(ex);
        if (!grad_out) fail(HARPIA_ERR_ARG, "grad_out is NULL");
        if (!sigma || !radius) fail(HARPIA_ERR_ARG, "sigma / radius is NULL");
        for (int a = 0; a < 3; ++a) {
            if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) fail(HARPIA_ERR_ARG, "sigma must be finite and > 0");
            if (radius[a] < 0 || radius[a] > kMaxGaussRadius)
                fail(HARPIA_ERR_ARG, "radius must be in [0, " + std::to_string(kMaxGaussRadius) + "]");
        }
        if (grad_sigma && !x) fail(HARPIA_ERR_ARG, "x is NULL (needed for grad_sigma)");
        if (grad_sigma && !valid_dtype(x_t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
        if (!grad_in && !grad_sigma) return;
        const int64_t nv = voxels(shape);
        if (grad_in) check_alias(grad_out, nv * 4, grad_in, nv * 4);
        if (grad_in && x) check_alias(x, nv * dtype_size(x_t), grad_in, nv * 4);
        reset_alloc_counter();
        if (!is_device_pointer(grad_out) || (grad_in && !is_device_pointer(grad_in)) ||
            (grad_sigma && !is_device_pointer(x)))
            fail(HARPIA_ERR_UNSUPPORTED, "the backward runs on device-resident volumes");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const int r[3] = {radius[0], radius[1], radius[2]};
        const Region g_reg = whole_region(grad_out, shape);
        bool allocated = false;
        DevBuf scratch, partials, dsig, dvol;
        if (grad_in) {
            // adjoint of the reflect-boundary Gaussian = the same Gaussian
            GaussTaps taps;
            make_gauss_taps_r(sigma, r, taps);
            const ChunkArgs a = make_chunk_args(g_reg, whole_region(grad_in, shape), shape);
            const size_t need = gaussian_scratch_bytes(shape, r, gauss_slices_fit(shape));
            if (need) {
                scratch.alloc(need);
                allocated = true;
            }
            if (!launch_gaussian(a, HARPIA_F32, HARPIA_F32, taps, s, scratch.p, need))
                fail(HARPIA_ERR_UNSUPPORTED, "no Gaussian kernel for these radii");
            check_hip(hipGetLastError(), "kernel launch");
        }
        if (grad_sigma) {
            // HARPIA_F_SIGMA_SUM: one value, the sum of the three axis terms
            const bool sum = ex && (ex->flags & HARPIA_F_SIGMA_SUM);
            const int n_sig = sum ? 1 : 3;
            const bool dev_out = is_device_pointer(grad_sigma);
            double *dst = grad_sigma;
            if (!dev_out) {
                dsig.alloc(3 * sizeof(double));
                dst = static_cast<double *>(dsig.p);
            }
            const Region x_reg = whole_region(x, shape);
            GaussTaps wt3, dt3;
            make_gauss_taps_r(sigma, r, wt3);
            make_gauss_dtaps3(sigma, r, dt3);
            const bool one_pass = r[0] == r[1] && r[1] == r[2] && r[0] >= 1 && r[0] <= kGaussFusedMaxR &&
                                  shape[1] * shape[2] < ((int64_t)1 << 31);
            if (one_pass) {
                // all three terms from one read of x and g
                partials.alloc((size_t)(3 * gauss_sigma3_blocks_bound(shape)) * sizeof(float));
                float *part = static_cast<float *>(partials.p);
                const int64_t nb = launch_gauss_sigma3(x, x_t, static_cast<const float *>(grad_out), shape, wt3, dt3,
                                                       s, part);
                if (nb < 0) fail(HARPIA_ERR_UNSUPPORTED, "no fused sigma-gradient kernel for these radii");
                check_hip(hipGetLastError(), "kernel launch");
                // the three terms' partials are contiguous: their sum is one
                // reduction over all of them
                for (int axis = 0; axis < n_sig; ++axis) {
                    launch_reduce_f64(part + axis * nb, sum ? 3 * nb : nb, dst + axis, false, s);
                    check_hip(hipGetLastError(), "kernel launch");
                }
            }
            for (int axis = 0; axis < 3 && !one_pass; ++axis) {
                GaussTaps dt;
                make_gauss_dtaps_r(sigma, r, axis, dt);
                // unfused: the derivative volume, then its dot with g
                if (!dvol.p) {
                    dvol.alloc((size_t)nv * sizeof(float));
                    const size_t need = gaussian_scratch_bytes(shape, r, false);
                    if (need && !scratch.p) scratch.alloc(need);
                }
                const Region d_reg = whole_region(dvol.p, shape);
                const ChunkArgs ad = make_chunk_args(x_reg, d_reg, shape);
                if (!launch_gaussian(ad, x_t, HARPIA_F32, dt, s, scratch.p, gaussian_scratch_bytes(shape, r, false)))
                    fail(HARPIA_ERR_UNSUPPORTED, "no Gaussian kernel for these radii");
                const int64_t max_blocks = 4096;
                if (!partials.p) partials.alloc((size_t)max_blocks * sizeof(float));
                const int64_t nb = launch_dot_partials(d_reg, g_reg, static_cast<float *>(partials.p), max_blocks, s);
                check_hip(hipGetLastError(), "kernel launch");
                launch_reduce_f64(static_cast<const float *>(partials.p), nb, dst + (sum ? 0 : axis), sum && axis > 0,
                                  s);
                check_hip(hipGetLastError(), "kernel launch");
            }
            if (!dev_out)
                check_hip(hipMemcpyAsync(grad_sigma, dst, n_sig * sizeof(double), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
            allocated = true;
        }
        if (allocated) check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    });
}

}  // extern "C"

namespace harpia {
namespace {

// Device scratch of harpia_gaussian3d_backward_noalloc: a 256-byte header
// for the sigma-gradient values (host destinations are copied from there)
// followed by the FP32 workgroup partials of the sigma-gradient kernel.
// Each GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` only names the symbol: its device address comes
// from hipGetSymbolAddress, looked up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
constexpr size_t kNoAllocHeaderBytes = 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxScratchDevices];

// Device address of the current device's copy of `scratch`.
unsigned char *device_scratch()
{
    int dev = -1;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) fail(HARPIA_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

}  // namespace
}  // namespace harpia

extern "C" {

harpia_status harpia_gaussian3d_backward_noalloc(const void *x, harpia_dtype x_t, const void *grad_out,
                                                 void *grad_in, const int64_t shape[3], const double sigma[3],
                                                 const int32_t radius[3], double *grad_sigma, const harpia_exec *ex)
{
    return guarded([&] {
        check_shape(shape);
        check_exec(ex);
        if (!grad_out) fail(HARPIA_ERR_ARG, "grad_out is NULL");
        if (!sigma || !radius) fail(HARPIA_ERR_ARG, "sigma / radius is NULL");
        for (int a = 0; a < 3; ++a) {
            if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) fail(HARPIA_ERR_ARG, "sigma must be finite and > 0");
            if (radius[a] < 0 || radius[a] > kMaxGaussRadius)
                fail(HARPIA_ERR_ARG, "radius must be in [0, " + std::to_string(kMaxGaussRadius) + "]");
        }
        if (grad_sigma && !x) fail(HARPIA_ERR_ARG, "x is NULL (needed for grad_sigma)");
        if (grad_sigma && !valid_dtype(x_t)) fail(HARPIA_ERR_DTYPE, "unsupported dtype");
        if (!grad_in && !grad_sigma) return;
        const int64_t nv = voxels(shape);
        if (grad_in) check_alias(grad_out, nv * 4, grad_in, nv * 4);
        if (grad_in && x) check_alias(x, nv * dtype_size(x_t), grad_in, nv * 4);
        reset_alloc_counter();  // the test hook then fails any allocation of this call
        if (!is_device_pointer(grad_out) || (grad_in && !is_device_pointer(grad_in)) ||
            (grad_sigma && !is_device_pointer(x)))
            fail(HARPIA_ERR_UNSUPPORTED, "the backward runs on device-resident volumes");
        const int r[3] = {radius[0], radius[1], radius[2]};
        // only the single-launch kernels, which need no scratch volume
        if (!(r[0] == r[1] && r[1] == r[2] && r[0] >= 1 && r[0] <= kGaussFusedMaxR) ||
            shape[1] * shape[2] >= ((int64_t)1 << 31) || !gauss_slices_fit(shape))
            fail(HARPIA_ERR_UNSUPPORTED, "the no-allocation backward needs equal radii in [1, " +
                                             std::to_string(kGaussFusedMaxR) + "] and slices of < 2^31 voxels");
        const size_t part_bytes = (size_t)(3 * gauss_sigma3_blocks_bound(shape)) * sizeof(float);
        if (grad_sigma && kNoAllocHeaderBytes + part_bytes > kNoAllocScratchBytes)
            fail(HARPIA_ERR_ARG, "volume too large for the no-allocation scratch: " + std::to_string(part_bytes) +
                                     " bytes of partials, at most " +
                                     std::to_string(kNoAllocScratchBytes - kNoAllocHeaderBytes));
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        unsigned char *base = grad_sigma ? device_scratch() : nullptr;
        if (grad_in) {
            GaussTaps taps;
            make_gauss_taps_r(sigma, r, taps);
            const ChunkArgs a = make_chunk_args(whole_region(grad_out, shape), whole_region(grad_in, shape), shape);
            if (!launch_gaussian(a, HARPIA_F32, HARPIA_F32, taps, s, nullptr, 0))
                fail(HARPIA_ERR_UNSUPPORTED, "no fused Gaussian kernel for these radii");
            check_hip(hipGetLastError(), "kernel launch");
        }
        if (grad_sigma) {
            const bool sum = ex && (ex->flags & HARPIA_F_SIGMA_SUM);
            const int n_sig = sum ? 1 : 3;
            const bool dev_out = is_device_pointer(grad_sigma);
            double *dst = dev_out ? grad_sigma : reinterpret_cast<double *>(base);
            float *part = reinterpret_cast<float *>(base + kNoAllocHeaderBytes);
            GaussTaps wt3, dt3;
            make_gauss_taps_r(sigma, r, wt3);
            make_gauss_dtaps3(sigma, r, dt3);
            // every partial the reduction reads is written by this launch
            const int64_t nb = launch_gauss_sigma3(x, x_t, static_cast<const float *>(grad_out), shape, wt3, dt3, s,
                                                   part);
            if (nb < 0) fail(HARPIA_ERR_UNSUPPORTED, "no fused sigma-gradient kernel for these radii");
            check_hip(hipGetLastError(), "kernel launch");
            for (int axis = 0; axis < n_sig; ++axis) {
                launch_reduce_f64(part + axis * nb, sum ? 3 * nb : nb, dst + axis, false, s);
                check_hip(hipGetLastError(), "kernel launch");
            }
            if (!dev_out) {
                check_hip(hipMemcpyAsync(grad_sigma, dst, n_sig * sizeof(double), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
                check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
            }
        }
    });
}

harpia_status harpia_morph3d_backward(const void *in, harpia_dtype t, const void *grad_out, void *grad_in,
                                      const int64_t shape[3], harpia_morph_op op, harpia_se se,
                                      const int32_t radius[3], const harpia_exec *ex)
{
    return guarded([&] {
        if (!in || !grad_out || !grad_in) fail(HARPIA_ERR_ARG, "in / grad_out / grad_in is NULL");
        check_shape(shape);
        check_exec(ex);
        if (op != HARPIA_ERODE && op != HARPIA_DILATE) fail(HARPIA_ERR_ARG, "unknown morphology op");
        const MorphArgs m = check_morph(t, se, radius, std::nan(""), HARPIA_BORDER_REFLECT, nullptr);
        if (!morph_grad_supported((int)se, m.r))
            fail(HARPIA_ERR_UNSUPPORTED, "morphology gradient: box radii above 8 or ball radius above 4");
        const int64_t nv = voxels(shape);
        check_alias(grad_out, nv * 4, grad_in, nv * 4);
        check_alias(in, nv * dtype_size(t), grad_in, nv * 4);
        reset_alloc_counter();
        if (!is_device_pointer(in) || !is_device_pointer(grad_out) || !is_device_pointer(grad_in))
            fail(HARPIA_ERR_UNSUPPORTED, "the backward runs on device-resident volumes");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        DevBuf code;
        code.alloc((size_t)nv * sizeof(uint16_t));
        const ChunkArgs a1 = make_chunk_args(whole_region(in, shape), whole_region(code.p, shape), shape);
        if (!launch_argext(a1, t, (int)op, (int)se, m.r, static_cast<uint16_t *>(code.p), s))
            fail(HARPIA_ERR_UNSUPPORTED, "no argext kernel");
        check_hip(hipGetLastError(), "kernel launch");
        const ChunkArgs a2 = make_chunk_args(whole_region(grad_out, shape), whole_region(grad_in, shape), shape);
        if (!launch_gather(a2, static_cast<const uint16_t *>(code.p), (int)se, m.r, s))
            fail(HARPIA_ERR_UNSUPPORTED, "no gather kernel");
        check_hip(hipGetLastError(), "kernel launch");
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    });
}


// ------------------------------------------------------------------ batched

static void check_crops(const harpia_crop *crops, int32_t n, bool need_in, bool need_out, bool need_aux)
{
    if (!crops || n < 1) fail(HARPIA_ERR_ARG, "crops is NULL or n_crops < 1");
    for (int32_t i = 0; i < n; ++i) {
        const harpia_crop &c = crops[i];
        for (int a = 0; a < 3; ++a)
            if (c.shape[a] <= 0 || c.shape[a] > (1 << 24)) fail(HARPIA_ERR_ARG, "crop extents must be in [1, 2^24]");
        if ((double)c.shape[1] * (double)c.shape[2] >= 2147483648.0)
            fail(HARPIA_ERR_UNSUPPORTED, "crop slices must hold fewer than 2^31 voxels");
        if ((need_in && !c.in) || (need_out && !c.out) || (need_aux && !c.aux))
            fail(HARPIA_ERR_ARG, "crop pointer is NULL");
        if ((c.in && !is_device_pointer(c.in)) || (c.out && !is_device_pointer(c.out)) ||
            (c.aux && !is_device_pointer(c.aux)))
            fail(HARPIA_ERR_UNSUPPORTED, "batched calls take device-resident crops");
    }
}

// Descriptor of crops [first, first + count) with the given role mapping.
static BatchDesc make_desc(const harpia_crop *crops, int32_t first, int32_t count, int role)
{
    BatchDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n_crops = count;
    for (int32_t i = 0; i < count; ++i) {
        const harpia_crop &c = crops[first + i];
        BatchCrop &k = d.c[i];
        switch (role) {
        case 0: k.in = c.in; k.out = c.out; k.aux = c.aux; break;                 // forward
        case 1: k.in = c.aux; k.out = c.out; k.aux = nullptr; break;              // grad_in = G grad_out
        case 2: k.in = c.in; k.out = const_cast<void *>(c.aux); k.aux = nullptr; break;  // dot(G' x, grad_out)
        }
        for (int a = 0; a < 3; ++a) k.n[a] = (int32_t)c.shape[a];
    }
    return d;
}

size_t harpia_batch_workspace_bytes(const harpia_crop *crops, int32_t n_crops)
{
    // sigma-gradient partials (3 axes x the largest persistent grid per
    // launch x launches) and u16 argext codes of every crop
    if (!crops || n_crops < 1) return 0;
    const int64_t launches = (n_crops + kMaxBatch - 1) / kMaxBatch;
    size_t bytes = (size_t)(3 * launches * gauss_batched_max_partials()) * sizeof(float);
    bytes = (bytes + 255) / 256 * 256;
    for (int32_t i = 0; i < n_crops; ++i) {
        const size_t v = (size_t)(crops[i].shape[0] * crops[i].shape[1] * crops[i].shape[2]);
        bytes += (v * sizeof(uint16_t) + 255) / 256 * 256;
    }
    return bytes;
}

harpia_status harpia_gaussian3d_batched(const harpia_crop *crops, int32_t n_crops, harpia_dtype in_t,
                                        harpia_dtype out_t, const double sigma[3], double truncate,
                                        const harpia_exec *ex)
{
    return guarded([&] {
        check_exec(ex);
        if (in_t != HARPIA_F32 || out_t != HARPIA_F32) fail(HARPIA_ERR_DTYPE, "batched calls take float32");
        if (!sigma) fail(HARPIA_ERR_ARG, "sigma is NULL");
        check_crops(crops, n_crops, true, true, false);
        const Stage st = gauss_stage(in_t, out_t, sigma, truncate);
        if (!(st.r[0] == st.r[1] && st.r[1] == st.r[2]) || st.r[0] < 1 || st.r[0] > kGaussFusedMaxR)
            fail(HARPIA_ERR_UNSUPPORTED, "batched Gaussian needs equal radii in [1, 12]");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        for (int32_t f = 0; f < n_crops; f += kMaxBatch) {
            const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
            if (!launch_gauss_batched(make_desc(crops, f, cnt, 0), in_t, out_t, st.taps, s))
                fail(HARPIA_ERR_UNSUPPORTED, "no batched Gaussian kernel");
            check_hip(hipGetLastError(), "kernel launch");
        }
    });
}

harpia_status harpia_morph3d_batched(const harpia_crop *crops, int32_t n_crops, harpia_dtype t,
                                     harpia_morph_op op, harpia_se se, const int32_t radius[3],
                                     const harpia_exec *ex)
{
    return guarded([&] {
        check_exec(ex);
        if (t != HARPIA_F32) fail(HARPIA_ERR_DTYPE, "batched calls take float32");
        if (op != HARPIA_ERODE && op != HARPIA_DILATE) fail(HARPIA_ERR_ARG, "unknown morphology op");
        const MorphArgs m = check_morph(t, se, radius, std::nan(""), HARPIA_BORDER_REFLECT, nullptr);
        if (!(m.r[0] == m.r[1] && m.r[1] == m.r[2]) || m.r[0] < 1 || m.r[0] > 4)
            fail(HARPIA_ERR_UNSUPPORTED, "batched morphology needs equal radii in [1, 4]");
        check_crops(crops, n_crops, true, true, false);
        const bool both = crops[0].aux != nullptr;
        for (int32_t i = 0; i < n_crops; ++i)
            if ((crops[i].aux != nullptr) != both) fail(HARPIA_ERR_ARG, "aux must be set for all crops or none");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        for (int32_t f = 0; f < n_crops; f += kMaxBatch) {
            const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
            if (!launch_morph_batched(make_desc(crops, f, cnt, 0), t, (int)op, (int)se, m.r[0], both, s))
                fail(HARPIA_ERR_UNSUPPORTED, "no batched morphology kernel");
            check_hip(hipGetLastError(), "kernel launch");
        }
    });
}

harpia_status harpia_gaussian3d_backward_batched(const harpia_crop *crops, int32_t n_crops,
                                                 const double sigma[3], const int32_t radius[3],
                                                 double *grad_sigma, void *workspace, size_t workspace_bytes,
                                                 const harpia_exec *ex)
{
    return guarded([&] {
        check_exec(ex);
        if (!sigma || !radius) fail(HARPIA_ERR_ARG, "sigma / radius is NULL");
        for (int a = 0; a < 3; ++a)
            if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) fail(HARPIA_ERR_ARG, "sigma must be finite and > 0");
        if (!(radius[0] == radius[1] && radius[1] == radius[2]) || radius[0] < 1 || radius[0] > kGaussFusedMaxR)
            fail(HARPIA_ERR_UNSUPPORTED, "batched Gaussian needs equal radii in [1, 12]");
        check_crops(crops, n_crops, grad_sigma != nullptr, false, true);
        const bool want_in = crops[0].out != nullptr;
        for (int32_t i = 0; i < n_crops; ++i)
            if ((crops[i].out != nullptr) != want_in) fail(HARPIA_ERR_ARG, "out must be set for all crops or none");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const int r[3] = {radius[0], radius[1], radius[2]};
        if (want_in) {
            GaussTaps taps;
            make_gauss_taps_r(sigma, r, taps);
            for (int32_t f = 0; f < n_crops; f += kMaxBatch) {
                const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
                if (!launch_gauss_batched(make_desc(crops, f, cnt, 1), HARPIA_F32, HARPIA_F32, taps, s))
                    fail(HARPIA_ERR_UNSUPPORTED, "no batched Gaussian kernel");
                check_hip(hipGetLastError(), "kernel launch");
            }
        }
        if (grad_sigma) {
            if (!is_device_pointer(grad_sigma)) fail(HARPIA_ERR_ARG, "grad_sigma must be a device pointer");
            const int64_t launches = (n_crops + kMaxBatch - 1) / kMaxBatch;
            const size_t need = (size_t)(3 * launches * gauss_batched_max_partials()) * sizeof(float);
            if (!workspace || workspace_bytes < need) fail(HARPIA_ERR_ARG, "workspace too small");
            if (!is_device_pointer(workspace)) fail(HARPIA_ERR_ARG, "workspace must be device memory");
            // all three terms in one pass per launch of up to 64 crops; each
            // launch's partials are reduced into grad_sigma in launch order
            GaussTaps wt3, dt3;
            make_gauss_taps_r(sigma, r, wt3);
            make_gauss_dtaps3(sigma, r, dt3);
            float *part = static_cast<float *>(workspace);
            for (int32_t f = 0, l = 0; f < n_crops; f += kMaxBatch, ++l) {
                const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
                float *pl = part + (int64_t)l * 3 * gauss_batched_max_partials();
                const int64_t grid = launch_gauss_sigma3_batched(make_desc(crops, f, cnt, 2), wt3, dt3, s, pl);
                if (grid < 0) fail(HARPIA_ERR_UNSUPPORTED, "no batched sigma-gradient kernel");
                check_hip(hipGetLastError(), "kernel launch");
                if (ex && (ex->flags & HARPIA_F_SIGMA_SUM)) {
                    launch_reduce_f64(pl, 3 * grid, grad_sigma, l > 0, s);
                    check_hip(hipGetLastError(), "kernel launch");
                }
                for (int axis = 0; axis < 3 && !(ex && (ex->flags & HARPIA_F_SIGMA_SUM)); ++axis) {
                    launch_reduce_f64(pl + axis * grid, grid, grad_sigma + axis, l > 0, s);
                    check_hip(hipGetLastError(), "kernel launch");
                }
            }
        }
    });
}

// u16 extremum codes of every crop, after the sigma-gradient partials in a
// batch workspace (layout of harpia_batch_workspace_bytes).
static std::vector<void *> batch_codes(const harpia_crop *crops, int32_t n_crops, void *workspace)
{
    const int64_t launches = (n_crops + kMaxBatch - 1) / kMaxBatch;
    size_t off = ((size_t)(3 * launches * gauss_batched_max_partials()) * sizeof(float) + 255) / 256 * 256;
    std::vector<void *> codes(n_crops);
    for (int32_t i = 0; i < n_crops; ++i) {
        codes[i] = static_cast<char *>(workspace) + off;
        const size_t v = (size_t)(crops[i].shape[0] * crops[i].shape[1] * crops[i].shape[2]);
        off += (v * sizeof(uint16_t) + 255) / 256 * 256;
    }
    return codes;
}

static MorphArgs check_batch_morph(const harpia_crop *crops, int32_t n_crops, harpia_morph_op op, harpia_se se,
                                   const int32_t radius[3], void *workspace, size_t workspace_bytes, bool need_in,
                                   bool need_aux)
{
    if (op != HARPIA_ERODE && op != HARPIA_DILATE) fail(HARPIA_ERR_ARG, "unknown morphology op");
    const MorphArgs m = check_morph(HARPIA_F32, se, radius, std::nan(""), HARPIA_BORDER_REFLECT, nullptr);
    if (!morph_grad_supported((int)se, m.r))
        fail(HARPIA_ERR_UNSUPPORTED, "morphology gradient: box radii above 8 or ball radius above 4");
    check_crops(crops, n_crops, need_in, true, need_aux);
    const size_t need = harpia_batch_workspace_bytes(crops, n_crops);
    if (!workspace || workspace_bytes < need) fail(HARPIA_ERR_ARG, "workspace too small");
    if (!is_device_pointer(workspace)) fail(HARPIA_ERR_ARG, "workspace must be device memory");
    return m;
}

harpia_status harpia_morph3d_forward_batched(const harpia_crop *crops, int32_t n_crops, harpia_morph_op op,
                                             harpia_se se, const int32_t radius[3], void *workspace,
                                             size_t workspace_bytes, const harpia_exec *ex)
{
    return guarded([&] {
        check_exec(ex);
        const MorphArgs m = check_batch_morph(crops, n_crops, op, se, radius, workspace, workspace_bytes, true, false);
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const std::vector<void *> codes = batch_codes(crops, n_crops, workspace);
        for (int32_t f = 0; f < n_crops; f += kMaxBatch) {
            const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
            // one pass: out = the extremum, aux = its code
            BatchDesc d = make_desc(crops, f, cnt, 0);
            for (int32_t i = 0; i < cnt; ++i) d.c[i].aux = codes[f + i];
            if (!launch_argext_batched(d, HARPIA_F32, (int)op, (int)se, m.r, s))
                fail(HARPIA_ERR_UNSUPPORTED, "no batched argext kernel");
            check_hip(hipGetLastError(), "kernel launch");
        }
    });
}

harpia_status harpia_morph3d_backward_batched(const harpia_crop *crops, int32_t n_crops, harpia_morph_op op,
                                              harpia_se se, const int32_t radius[3], void *workspace,
                                              size_t workspace_bytes, const harpia_exec *ex)
{
    return guarded([&] {
        check_exec(ex);
        const bool reuse = ex && (ex->flags & HARPIA_F_REUSE_CODES);
        const MorphArgs m = check_batch_morph(crops, n_crops, op, se, radius, workspace, workspace_bytes, !reuse, true);
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const std::vector<void *> codes = batch_codes(crops, n_crops, workspace);
        for (int32_t f = 0; f < n_crops; f += kMaxBatch) {
            const int32_t cnt = std::min<int32_t>(kMaxBatch, n_crops - f);
            BatchDesc d = make_desc(crops, f, cnt, 0);
            if (!reuse) {
                // argext: in = forward input, aux = codes (no values)
                for (int32_t i = 0; i < cnt; ++i) {
                    d.c[i].aux = codes[f + i];
                    d.c[i].out = nullptr;
                }
                if (!launch_argext_batched(d, HARPIA_F32, (int)op, (int)se, m.r, s))
                    fail(HARPIA_ERR_UNSUPPORTED, "no batched argext kernel");
                check_hip(hipGetLastError(), "kernel launch");
            }
            // gather: in = upstream gradient, aux = codes, out = grad_in
            for (int32_t i = 0; i < cnt; ++i) {
                d.c[i].in = crops[f + i].aux;
                d.c[i].aux = codes[f + i];
                d.c[i].out = crops[f + i].out;
            }
            if (!launch_gather_batched(d, (int)se, m.r, s)) fail(HARPIA_ERR_UNSUPPORTED, "no batched gather kernel");
            check_hip(hipGetLastError(), "kernel launch");
        }
    });
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner

namespace harpia {
namespace {

// Runs `call` under every candidate tile of `fam`, keeps the fastest (a
// candidate must beat the heuristic, candidate 0, by 2 %), records it for the
// workloads the forced launches saw and appends a report entry.
template <class Call>
void tune_family(int fam, hipStream_t s, int reps, Call call, harpia_tune_report *rep)
{
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    check_hip(hipEventCreate(&ev.a), "hipEventCreate");
    check_hip(hipEventCreate(&ev.b), "hipEventCreate");
    struct Unforce {
        ~Unforce() { tune_force(0, -1); }
    } unforce;
    auto run = [&] {
        const harpia_status st = call();
        if (st != HARPIA_OK) fail(st, harpia_last_error());
    };
    const int n = tune_candidates(fam);
    int best = 0;
    float best_ms = 0.f, heur_ms = 0.f;
    // each candidate: one warm-up, then the fastest of `reps` runs timed one
    // by one (the minimum is far less noisy than a mean on a shared device)
    auto time_one = [&]() -> float {
        check_hip(hipEventRecord(ev.a, s), "hipEventRecord");
        run();
        check_hip(hipEventRecord(ev.b, s), "hipEventRecord");
        check_hip(hipEventSynchronize(ev.b), "hipEventSynchronize");
        float ms = 0.f;
        check_hip(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
        return ms;
    };
    for (int i = 0; i < n; ++i) {
        tune_force(fam, i);
        run();  // warm-up
        float ms = time_one();
        for (int k = 1; k < reps; ++k) ms = std::min(ms, time_one());
        if (i == 0) {
            heur_ms = best_ms = ms;
        } else if (ms < best_ms && ms < 0.98f * heur_ms) {
            best_ms = ms;
            best = i;
        }
    }
    // one more run under the winner collects the workload keys to record
    tune_force(fam, best);
    run();
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    const Tile t = tune_candidate(fam, best);
    tune_record_seen(fam, t);
    if (rep && rep->n < (int32_t)(sizeof(rep->e) / sizeof(rep->e[0]))) {
        harpia_tune_entry &e = rep->e[rep->n++];
        std::memset(&e, 0, sizeof(e));
        std::strncpy(e.kernel, tune_family_name(fam), sizeof(e.kernel) - 1);
        e.tile[0] = t.tx;
        e.tile[1] = t.ty;
        e.tile[2] = t.tz;
        e.candidates = n;
        e.ms_heuristic = heur_ms;
        e.ms_best = best_ms;
    }
}

int tune_reps(int32_t reps) { return reps > 0 ? (reps < 100 ? reps : 100) : 3; }

}  // namespace
}  // namespace harpia

extern "C" {

using namespace harpia;

harpia_status harpia_autotune_gaussian3d(const void *in, harpia_dtype in_t, void *out, harpia_dtype out_t,
                                         const int64_t shape[3], const double sigma[3], double truncate,
                                         int32_t reps, const harpia_exec *ex, harpia_tune_report *report)
{
    return guarded([&] {
        if (report) report->n = 0;
        if (!in || !out) fail(HARPIA_ERR_ARG, "in / out is NULL");
        if (!is_device_pointer(in) || !is_device_pointer(out))
            fail(HARPIA_ERR_UNSUPPORTED, "the autotuner runs on device-resident volumes");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        tune_family(TF_GAUSS, s, tune_reps(reps), [&] {
            return harpia_gaussian3d(in, in_t, out, out_t, shape, sigma, truncate, HARPIA_BORDER_REFLECT, ex);
        }, report);
    });
}

harpia_status harpia_autotune_erode_dilate3d(const void *in, void *out_erode, void *out_dilate, harpia_dtype t,
                                             const int64_t shape[3], harpia_se se, const int32_t radius[3],
                                             double threshold, int32_t reps, const harpia_exec *ex,
                                             harpia_tune_report *report)
{
    return guarded([&] {
        if (report) report->n = 0;
        if (!in || !out_erode || !out_dilate) fail(HARPIA_ERR_ARG, "in / out is NULL");
        if (!is_device_pointer(in) || !is_device_pointer(out_erode) || !is_device_pointer(out_dilate))
            fail(HARPIA_ERR_UNSUPPORTED, "the autotuner runs on device-resident volumes");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const bool binary = !std::isnan(threshold) || (ex && (ex->flags & HARPIA_F_BINARY));
        tune_family(binary ? TF_BINARY : TF_GRAY, s, tune_reps(reps), [&] {
            return harpia_erode_dilate3d(in, out_erode, out_dilate, t, shape, se, radius, threshold,
                                         HARPIA_BORDER_REFLECT, ex);
        }, report);
    });
}

harpia_status harpia_autotune_gauss_dilate_batched(const harpia_crop *crops, int32_t n_crops, const double sigma[3],
                                                   const int32_t gauss_radius[3], harpia_se se,
                                                   const int32_t morph_radius[3], void *workspace,
                                                   size_t workspace_bytes, int32_t reps, const harpia_exec *ex,
                                                   harpia_tune_report *report)
{
    return guarded([&] {
        if (report) report->n = 0;
        check_crops(crops, n_crops, true, true, true);
        if (!sigma || !gauss_radius || !morph_radius) fail(HARPIA_ERR_ARG, "sigma / radius is NULL");
        hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
        const int nr = std::max(1, tune_reps(reps) - 1);
        // the Gaussian's truncate is chosen so that it resolves to gauss_radius
        const double trunc = ((double)gauss_radius[0] + 0.25) / sigma[0];
        std::vector<harpia_crop> fwd(crops, crops + n_crops), mor(n_crops), bwd(n_crops), dot(n_crops);
        for (int32_t i = 0; i < n_crops; ++i) {
            // x -> A (Gaussian), A -> B (dilation), subgradient of the
            // dilation of A with upstream x into B, sigma-gradient with x and A
            mor[i] = harpia_crop{crops[i].out, const_cast<void *>(crops[i].aux), nullptr, {0, 0, 0}};
            bwd[i] = harpia_crop{crops[i].out, const_cast<void *>(crops[i].aux), crops[i].in, {0, 0, 0}};
            dot[i] = harpia_crop{crops[i].in, nullptr, crops[i].out, {0, 0, 0}};
            for (int a = 0; a < 3; ++a) mor[i].shape[a] = bwd[i].shape[a] = dot[i].shape[a] = crops[i].shape[a];
        }
        tune_family(TF_GAUSS_BATCHED, s, nr, [&] {
            return harpia_gaussian3d_batched(fwd.data(), n_crops, HARPIA_F32, HARPIA_F32, sigma, trunc, ex);
        }, report);
        tune_family(TF_GRAY_BATCHED, s, nr, [&] {
            return harpia_morph3d_batched(mor.data(), n_crops, HARPIA_F32, HARPIA_DILATE, se, morph_radius, ex);
        }, report);
        if (se == HARPIA_SE_BOX) {
            for (int fam : {TF_ARGEXT_BOX, TF_GATHER_BOX})
                tune_family(fam, s, nr, [&] {
                    return harpia_morph3d_backward_batched(bwd.data(), n_crops, HARPIA_DILATE, se, morph_radius,
                                                           workspace, workspace_bytes, ex);
                }, report);
        }
        double *gs = nullptr;
        check_hip(hipMalloc(&gs, 3 * sizeof(double)), "hipMalloc");
        struct Free {
            double *p;
            ~Free() { (void)hipFree(p); }
        } free_gs{gs};
        tune_family(TF_GAUSS_DOT_BATCHED, s, nr, [&] {
            return harpia_gaussian3d_backward_batched(dot.data(), n_crops, sigma, gauss_radius, gs, workspace,
                                                      workspace_bytes, ex);
        }, report);
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    });
}

harpia_status harpia_tune_clear(void)
{
    return guarded([&] { tune_clear(); });
}

int64_t harpia_tune_entries(void) { return tune_size(); }

harpia_status harpia_tune_save(const char *path)
{
    return guarded([&] {
        if (!path) fail(HARPIA_ERR_ARG, "path is NULL");
        if (!tune_save(path)) fail(HARPIA_ERR_ARG, std::string("cannot write ") + path);
    });
}

harpia_status harpia_tune_load(const char *path)
{
    return guarded([&] {
        if (!path) fail(HARPIA_ERR_ARG, "path is NULL");
        if (!tune_load(path)) fail(HARPIA_ERR_ARG, std::string("cannot read a tune cache from ") + path);
    });
}

}  // extern "C"
