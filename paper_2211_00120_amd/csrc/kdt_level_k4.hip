// kdt_level_k4.hip -- level-pass kernels for k = 4.
#include "kdt_level.h"

namespace kdt {
template void launch_level_pass_k<4>(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st);
}  // namespace kdt
