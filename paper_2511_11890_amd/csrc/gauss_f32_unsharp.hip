// Fused Gaussian with the unsharp-mask epilogue, float -> float.
#include "gauss_impl.h"

namespace harpia {
namespace gauss_detail {
template bool fused_family_run<float, float, 1>(int, const ChunkArgs &, const GaussTaps &, hipStream_t);
}  // namespace gauss_detail
}  // namespace harpia
