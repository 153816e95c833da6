// Erosion / dilation kernels instantiated for bf16_t input.
#include "morph_impl.h"

namespace harpia {
template bool morph_run<bf16_t>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
}  // namespace harpia
