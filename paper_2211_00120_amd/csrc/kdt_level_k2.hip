// kdt_level_k2.hip -- level-pass kernels for k = 2.
#include "kdt_level.h"

namespace kdt {
template void launch_level_pass_k<2>(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st);
}  // namespace kdt
