// Erosion / dilation kernels instantiated for uint8_t input.
#include "morph_impl.h"

namespace harpia {
template bool morph_run<uint8_t>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
}  // namespace harpia
