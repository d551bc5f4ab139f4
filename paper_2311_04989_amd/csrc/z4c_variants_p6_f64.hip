// z4c_variants_p6_f64.hip -- instantiations of the tile kernels (see z4c_tile.h).
#include "z4c_tile.h"

namespace z4c {

hipError_t launch_p6_f64(int mode, int tx, int ty, int tz, int w, const StageArgs &a,
                         hipStream_t s)
{
    if (mode == MODE_CONS) {
        if (ty == 4)
            return launch_cons<6, 8, 4, 8>(a, s);
        if (tz == 4)
            return launch_cons<6, 8, 8, 4>(a, s);
        return launch_cons<6, 8, 8, 8>(a, s);
    }
    if (tx == 8 && ty == 8 && tz == 8 && w == 2)
        return launch_variant<6, 8, 8, 8, 2, double>(mode, a, s);
    if (tx == 8 && ty == 8 && tz == 4 && w == 2)
        return launch_variant<6, 8, 8, 4, 2, double>(mode, a, s);
    if (tx == 8 && ty == 8 && tz == 4 && w == 1)
        return launch_variant<6, 8, 8, 4, 1, double>(mode, a, s);
    if (tx == 8 && ty == 4 && tz == 8 && w == 1)
        return launch_variant<6, 8, 4, 8, 1, double>(mode, a, s);
    return hipErrorInvalidValue;
}

}  // namespace z4c
