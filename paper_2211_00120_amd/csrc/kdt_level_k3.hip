// kdt_level_k3.hip -- level-pass kernels for k = 3.
#include "kdt_level.h"

namespace kdt {
template void launch_level_pass_k<3>(const LevelPassArgs& a, uint32_t tiles, bool last, bool widest, hipStream_t st);
}  // namespace kdt
