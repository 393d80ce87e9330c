// Moment-pass tile kernels, FP64 path, orders L = 21..26.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f64_c(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(double, 21)
        TCM_TILE_CASE(double, 22)
        TCM_TILE_CASE(double, 23)
        TCM_TILE_CASE(double, 24)
        TCM_TILE_CASE(double, 25)
        TCM_TILE_CASE(double, 26)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
