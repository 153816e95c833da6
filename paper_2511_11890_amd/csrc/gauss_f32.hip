// Gaussian kernels instantiated for float -> float.
#include "gauss_impl.h"

namespace harpia {
template bool gauss_run<float, float>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
template int64_t gauss_sigma3_run<float>(const float *, const float *, const int64_t *, const GaussTaps &,
                                          const GaussTaps &, hipStream_t, float *);
template int64_t gauss_sigma3_batched_run<float>(const BatchDesc &, const GaussTaps &, const GaussTaps &,
                                                 hipStream_t, float *);
template bool gauss_batched_run<float, float>(const BatchDesc &, const GaussTaps &, hipStream_t);
}  // namespace harpia
