// kdt_level_k1.hip -- level-pass kernels for k = 1.
#include "kdt_level.h"

namespace kdt {
template void launch_level_pass_k<1>(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st);
}  // namespace kdt
