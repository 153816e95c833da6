// Fused Gaussian with odd (first-derivative) taps on some axes, float ->
// float: the mixed components of the Hessian.
#include "gauss_impl.h"

namespace harpia {
namespace gauss_detail {
template bool fused_family_run<float, float, 2>(int, const ChunkArgs &, const GaussTaps &, hipStream_t);
}  // namespace gauss_detail
}  // namespace harpia
