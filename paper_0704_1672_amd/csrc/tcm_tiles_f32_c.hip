// Moment-pass tile kernels, FP32 compensated path, orders L = 21..26.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f32_c(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(float, 21)
        TCM_TILE_CASE(float, 22)
        TCM_TILE_CASE(float, 23)
        TCM_TILE_CASE(float, 24)
        TCM_TILE_CASE(float, 25)
        TCM_TILE_CASE(float, 26)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
