// Binary erosion / dilation kernels instantiated for float input.
#include "morph_impl.h"

namespace harpia {
namespace morph_detail {
template bool bits_run<float>(int, int, bool, const ChunkArgs &, const MorphSpec &, const Out2 &, float, hipStream_t);
}  // namespace morph_detail
}  // namespace harpia
