// Erosion / dilation kernels instantiated for float input.
#include "morph_impl.h"

namespace harpia {
template bool morph_run<float>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
template bool morph_batched_run<float>(const BatchDesc &, int, int, int, bool, hipStream_t);
}  // namespace harpia
