// Erosion / dilation kernels instantiated for _Float16 input.
#include "morph_impl.h"

namespace harpia {
template bool morph_run<_Float16>(const ChunkArgs &, const MorphSpec &, bool, const Region *, float, hipStream_t);
}  // namespace harpia
