// z4c_variants_naive.hip -- instantiations of the naive-FP32 right-hand side
// (see z4c_tile.h): every staged sample rounded to float before the stencil
// differences, order 6, every supported launch shape.
#include "z4c_tile.h"

namespace z4c {

hipError_t launch_naive(int fd_order, int tx, int ty, int tz, int w, const StageArgs &a,
                        hipStream_t s)
{
    if (fd_order != 6)
        return hipErrorInvalidValue;
    if (tx == 8 && ty == 8 && tz == 8 && w == 2)
        return launch_variant_naive<6, 8, 8, 8, 2>(a, s);
    if (tx == 8 && ty == 8 && tz == 4 && w == 2)
        return launch_variant_naive<6, 8, 8, 4, 2>(a, s);
    if (tx == 8 && ty == 8 && tz == 4 && w == 1)
        return launch_variant_naive<6, 8, 8, 4, 1>(a, s);
    if (tx == 8 && ty == 4 && tz == 8 && w == 1)
        return launch_variant_naive<6, 8, 4, 8, 1>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace z4c
