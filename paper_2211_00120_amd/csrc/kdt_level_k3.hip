// kdt_level_k3.hip -- split-pass kernels for k = 3 (one file per k, so the
// instantiations compile in parallel).
#include "kdt_level.h"

namespace kdt {
template void launch_level_pivot_k<3>(const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st);
template void launch_level_part_k<3>(const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st);
}  // namespace kdt
