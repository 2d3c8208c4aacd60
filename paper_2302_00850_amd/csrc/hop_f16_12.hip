// Hop kernel instantiations: F16 spinors, F16_12 links.
#include "hop_impl.h"

namespace cola {

hipError_t hop_launch_f16_12(const HopArgs &a, int rpt, int grid, int block, hipStream_t st) {
    return hop_launch_fmt<SpinorFmt::F16, LinkFmt::F16_12, float>(a, rpt, grid, block, st);
}

}  // namespace cola
