// Moment-pass tile kernels, FP64 path, orders L = 13..20.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f64_b(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(double, 13)
        TCM_TILE_CASE(double, 14)
        TCM_TILE_CASE(double, 15)
        TCM_TILE_CASE(double, 16)
        TCM_TILE_CASE(double, 17)
        TCM_TILE_CASE(double, 18)
        TCM_TILE_CASE(double, 19)
        TCM_TILE_CASE(double, 20)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
