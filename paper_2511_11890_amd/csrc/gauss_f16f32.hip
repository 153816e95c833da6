// Gaussian kernels instantiated for _Float16 -> float.
#include "gauss_impl.h"

namespace harpia {
template bool gauss_run<_Float16, float>(const ChunkArgs &, const GaussTaps &, hipStream_t, void *, size_t);
}  // namespace harpia
