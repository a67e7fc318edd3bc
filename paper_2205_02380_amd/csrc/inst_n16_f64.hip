// Kernel instantiations: CHASM_SHAPES_N16_F64.
#include "chasm_launch.hpp"

namespace chasm {
CHASM_SHAPES_N16_F64(CHASM_INSTANTIATE)
}  // namespace chasm
