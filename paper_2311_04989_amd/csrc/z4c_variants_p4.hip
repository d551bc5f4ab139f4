// z4c_variants_p4.hip -- instantiations of the tile kernels (see z4c_tile.h).
#include "z4c_tile.h"

namespace z4c {

hipError_t launch_p4(int mode, int arith, int tx, int ty, int tz, int w, const StageArgs &a,
                     hipStream_t s)
{
    (void)w;
    if (mode == MODE_CONS) {
        if (tz == 4)
            return launch_cons<4, 8, 8, 4>(a, s);
        return launch_cons<4, 8, 8, 8>(a, s);
    }
    if (tx == 8 && ty == 8 && tz == 8) {
        if (arith == Z4C_ARITH_FP32)
            return launch_variant<4, 8, 8, 8, 2, float>(mode, a, s);
        return launch_variant<4, 8, 8, 8, 2, double>(mode, a, s);
    }
    if (tx == 8 && ty == 8 && tz == 4) {
        if (arith == Z4C_ARITH_FP32)
            return launch_variant<4, 8, 8, 4, 2, float>(mode, a, s);
        return launch_variant<4, 8, 8, 4, 2, double>(mode, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace z4c
