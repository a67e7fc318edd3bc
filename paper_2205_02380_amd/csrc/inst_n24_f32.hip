// Kernel instantiations: CHASM_SHAPES_N24_F32.
#include "chasm_launch.hpp"

namespace chasm {
CHASM_SHAPES_N24_F32(CHASM_INSTANTIATE)
}  // namespace chasm
