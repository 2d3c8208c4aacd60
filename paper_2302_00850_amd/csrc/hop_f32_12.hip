// Hop kernel instantiations: F32 spinors, F32_12 links.
#include "hop_impl.h"

namespace cola {

hipError_t hop_launch_f32_12(const HopArgs &a, int rpt, int grid, int block, hipStream_t st) {
    return hop_launch_fmt<SpinorFmt::F32, LinkFmt::F32_12, float>(a, rpt, grid, block, st);
}

}  // namespace cola
