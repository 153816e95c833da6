// Gaussian kernels instantiated for uint16_t -> float.
#include "gauss_impl.h"

namespace harpia {
template bool gauss_run<uint16_t, float>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
template int64_t gauss_sigma3_run<uint16_t>(const uint16_t *, const float *, const int64_t *, const GaussTaps &,
                                          const GaussTaps &, hipStream_t, float *);
}  // namespace harpia
