// kdt_level_k2.hip -- split-pass kernels for k = 2 (one file per k, so the
// instantiations compile in parallel).
#include "kdt_level.h"

namespace kdt {
template void launch_level_pivot_k<2>(const LevelPivotArgs& a, uint32_t tiles, bool widest, hipStream_t st);
template void launch_level_part_k<2>(const LevelPartArgs& a, uint32_t tiles, bool widest, hipStream_t st);
}  // namespace kdt
