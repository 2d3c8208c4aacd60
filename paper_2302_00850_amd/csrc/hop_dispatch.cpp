// Dispatch of a hop launch to the translation unit of its precision.
#include "launch.h"

namespace cola {

hipError_t hop_launch_f64_18(const HopArgs &a, int rpt, int grid, int block, hipStream_t st);
hipError_t hop_launch_f64_12(const HopArgs &a, int rpt, int grid, int block, hipStream_t st);
hipError_t hop_launch_f32_12(const HopArgs &a, int rpt, int grid, int block, hipStream_t st);
hipError_t hop_launch_f16_12(const HopArgs &a, int rpt, int grid, int block, hipStream_t st);
hipError_t hop_launch_flic(const HopArgs &a, LinkFmt lf, int rpt, int grid, int block,
                           hipStream_t st);

hipError_t launch_hop(const HopArgs &a, LinkFmt lf, int rpt, int grid, int block,
                      hipStream_t st) {
    if (a.gauge_fat) return hop_launch_flic(a, lf, rpt, grid, block, st);
    switch (lf) {
        case LinkFmt::F64_18: return hop_launch_f64_18(a, rpt, grid, block, st);
        case LinkFmt::F64_12: return hop_launch_f64_12(a, rpt, grid, block, st);
        case LinkFmt::F32_12: return hop_launch_f32_12(a, rpt, grid, block, st);
        case LinkFmt::F16_12: return hop_launch_f16_12(a, rpt, grid, block, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace cola
