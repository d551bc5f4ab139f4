// z4c_variants_mon.hip -- instantiations of the stage kernel with the
// constraint monitor (FP64 arithmetic; see z4c_tile.h).
#include "z4c_tile.h"

namespace z4c {

hipError_t launch_monitor(int fd_order, int tx, int ty, int tz, int w, const StageArgs &a,
                          hipStream_t s)
{
    if (fd_order == 6) {
        if (tx == 8 && ty == 8 && tz == 8 && w == 2)
            return launch_variant_mon<6, 8, 8, 8, 2>(a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 2)
            return launch_variant_mon<6, 8, 8, 4, 2>(a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 1)
            return launch_variant_mon<6, 8, 8, 4, 1>(a, s);
        if (tx == 8 && ty == 4 && tz == 8 && w == 1)
            return launch_variant_mon<6, 8, 4, 8, 1>(a, s);
    } else if (fd_order == 4) {
        if (tx == 8 && ty == 8 && tz == 8 && w == 2)
            return launch_variant_mon<4, 8, 8, 8, 2>(a, s);
        if (tx == 8 && ty == 8 && tz == 4 && w == 2)
            return launch_variant_mon<4, 8, 8, 4, 2>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace z4c
