// Dispatch of one morphology step to the per-dtype kernel instantiations.
#include <cmath>

#include "common.h"
#include "batch.h"

namespace harpia {

template <typename T>
bool morph_run(const ChunkArgs &a, const MorphSpec &m, bool both, const Region *out2, float thr_f, hipStream_t s);

// Threshold in the f32 domain the kernels compare in, chosen so that
// (float)v > thr_f  <=>  v > t  exactly for every value v of dtype `t`:
// integers compare against floor(t); float types against the largest float
// not above t (no float lies between it and t).
float compare_threshold(harpia_dtype t, double thr)
{
    if (t == HARPIA_U8 || t == HARPIA_U16) {
        double f = std::floor(thr);
        if (f < -1.0) f = -1.0;
        if (f > 65536.0) f = 65536.0;
        return (float)f;
    }
    float f = (float)thr;
    if ((double)f > thr) f = std::nextafter(f, -INFINITY);
    return f;
}

bool launch_morph_ex(const ChunkArgs &a, harpia_dtype t, const MorphSpec &m, bool both, const Region *out2,
                     hipStream_t s)
{
    const float thr_f = m.has_threshold ? compare_threshold(t, m.threshold) : 0.f;
    switch (t) {
    case HARPIA_U8: return morph_run<uint8_t>(a, m, both, out2, thr_f, s);
    case HARPIA_U16: return morph_run<uint16_t>(a, m, both, out2, thr_f, s);
    case HARPIA_F32: return morph_run<float>(a, m, both, out2, thr_f, s);
    case HARPIA_F16: return morph_run<_Float16>(a, m, both, out2, thr_f, s);
    case HARPIA_BF16: return morph_run<bf16_t>(a, m, both, out2, thr_f, s);
    }
    return false;
}

template <typename T>
bool morph_batched_run(const BatchDesc &d, int op, int se, int r, bool both, hipStream_t s);

bool launch_morph_batched(const BatchDesc &d, harpia_dtype t, int op, int se, int r, bool both, hipStream_t s)
{
    if (t != HARPIA_F32) return false;
    return morph_batched_run<float>(d, op, se, r, both, s);
}

bool launch_morph(const ChunkArgs &a, harpia_dtype t, const MorphSpec &m, hipStream_t s)
{
    return launch_morph_ex(a, t, m, false, nullptr, s);
}

}  // namespace harpia
