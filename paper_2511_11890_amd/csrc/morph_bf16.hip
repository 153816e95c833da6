// Erosion / dilation kernels (grayscale) instantiated for bf16_t input.
#include "morph_impl.h"

namespace harpia {
namespace morph_detail {
extern template bool bits_run<bf16_t>(int, int, bool, const ChunkArgs &, const MorphSpec &, const Out2 &, float,
                                 hipStream_t);
}  // namespace morph_detail
template bool morph_run<bf16_t>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
}  // namespace harpia
