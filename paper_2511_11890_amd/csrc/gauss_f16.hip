// Gaussian kernels instantiated for _Float16 -> _Float16.
#include "gauss_impl.h"

namespace harpia {
template bool gauss_run<_Float16, _Float16>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
template int64_t gauss_sigma3_run<_Float16>(const _Float16 *, const float *, const int64_t *, const GaussTaps &,
                                          const GaussTaps &, hipStream_t, float *);
}  // namespace harpia
