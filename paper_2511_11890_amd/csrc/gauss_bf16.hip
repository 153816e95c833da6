// Gaussian kernels instantiated for bf16_t -> bf16_t.
#include "gauss_impl.h"

namespace harpia {
template bool gauss_run<bf16_t, bf16_t>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
template int64_t gauss_sigma3_run<bf16_t>(const bf16_t *, const float *, const int64_t *, const GaussTaps &,
                                          const GaussTaps &, hipStream_t, float *);
}  // namespace harpia
