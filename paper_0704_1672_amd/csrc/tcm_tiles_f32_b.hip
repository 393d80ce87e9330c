// Moment-pass tile kernels, FP32 compensated path, orders L = 13..20.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f32_b(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(float, 13)
        TCM_TILE_CASE(float, 14)
        TCM_TILE_CASE(float, 15)
        TCM_TILE_CASE(float, 16)
        TCM_TILE_CASE(float, 17)
        TCM_TILE_CASE(float, 18)
        TCM_TILE_CASE(float, 19)
        TCM_TILE_CASE(float, 20)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
