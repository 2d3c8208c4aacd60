// Hop kernel instantiations: F64 spinors, F64_18 links.
#include "hop_impl.h"

namespace cola {

hipError_t hop_launch_f64_18(const HopArgs &a, int rpt, int grid, int block, hipStream_t st) {
    return hop_launch_fmt<SpinorFmt::F64, LinkFmt::F64_18, double>(a, rpt, grid, block, st);
}

}  // namespace cola
