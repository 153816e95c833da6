// Erosion / dilation kernels (grayscale) instantiated for float input.
#include "morph_impl.h"

namespace harpia {
namespace morph_detail {
extern template bool bits_run<float>(int, int, bool, const ChunkArgs &, const MorphSpec &, const Out2 &, float,
                                 hipStream_t);
}  // namespace morph_detail
template bool morph_run<float>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
template bool morph_batched_run<float>(const BatchDesc &, int, int, int, bool, hipStream_t);
}  // namespace harpia
