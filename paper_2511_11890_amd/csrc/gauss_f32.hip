// Gaussian kernels instantiated for float -> float: plain smoothing and the
// single-volume sigma-gradient.  The unsharp and odd-tap families and the
// batched kernels are compiled in gauss_f32_*.hip (in parallel).
#include "gauss_impl.h"

namespace harpia {
namespace gauss_detail {
extern template bool fused_family_run<float, float, 1>(int, const ChunkArgs &, const GaussTaps &, hipStream_t);
extern template bool fused_family_run<float, float, 2>(int, const ChunkArgs &, const GaussTaps &, hipStream_t);
}  // namespace gauss_detail

template bool gauss_run<float, float>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
template int64_t gauss_sigma3_run<float>(const float *, const float *, const int64_t *, const GaussTaps &,
                                          const GaussTaps &, hipStream_t, float *);
}  // namespace harpia
