// Binary erosion / dilation kernels instantiated for uint8_t input.
#include "morph_impl.h"

namespace harpia {
namespace morph_detail {
template bool bits_run<uint8_t>(int, int, bool, const ChunkArgs &, const MorphSpec &, const Out2 &, float, hipStream_t);
}  // namespace morph_detail
}  // namespace harpia
