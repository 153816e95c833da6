// Batched Gaussian and batched sigma-gradient kernels, float32 crops.
#include "gauss_impl.h"

namespace harpia {
template int64_t gauss_sigma3_batched_run<float>(const BatchDesc &, const GaussTaps &, const GaussTaps &,
                                                 hipStream_t, float *);
template bool gauss_batched_run<float, float>(const BatchDesc &, const GaussTaps &, hipStream_t);
}  // namespace harpia
