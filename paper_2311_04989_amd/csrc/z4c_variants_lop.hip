// z4c_variants_lop.hip -- instantiations of the right-hand side and stage
// kernels with lopsided advection (FP64 arithmetic; see z4c_tile.h).
#include "z4c_tile.h"

namespace z4c {

hipError_t launch_lopsided(int mode, int fd_order, int tx, int ty, int tz, int w,
                           const StageArgs &a, hipStream_t s)
{
    if (fd_order == 6) {
        if (tx == 8 && ty == 8 && tz == 8 && w == 2)
            return launch_variant_lop<6, 8, 8, 8, 2>(mode, a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 2)
            return launch_variant_lop<6, 8, 8, 4, 2>(mode, a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 1)
            return launch_variant_lop<6, 8, 8, 4, 1>(mode, a, s);
        if (tx == 8 && ty == 4 && tz == 8 && w == 1)
            return launch_variant_lop<6, 8, 4, 8, 1>(mode, a, s);
    } else if (fd_order == 4) {
        if (tx == 8 && ty == 8 && tz == 8 && w == 2)
            return launch_variant_lop<4, 8, 8, 8, 2>(mode, a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 2)
            return launch_variant_lop<4, 8, 8, 4, 2>(mode, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace z4c
