// Hop kernel instantiations of the FLIC operator (thin and smeared links): FP64 spinors
// with 18- or 12-real links, FP32 spinors with 12-real links.
#include "hop_impl.h"

namespace cola {

hipError_t hop_launch_flic(const HopArgs &a, LinkFmt lf, int rpt, int grid, int block,
                           hipStream_t st) {
    switch (lf) {
        case LinkFmt::F64_18:
            return hop_launch_flic_fmt<SpinorFmt::F64, LinkFmt::F64_18, double>(a, rpt, grid,
                                                                               block, st);
        case LinkFmt::F64_12:
            return hop_launch_flic_fmt<SpinorFmt::F64, LinkFmt::F64_12, double>(a, rpt, grid,
                                                                               block, st);
        case LinkFmt::F32_12:
            return hop_launch_flic_fmt<SpinorFmt::F32, LinkFmt::F32_12, float>(a, rpt, grid,
                                                                              block, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cola
