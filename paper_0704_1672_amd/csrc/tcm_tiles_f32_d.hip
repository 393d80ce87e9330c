// Moment-pass tile kernels, FP32 compensated path, orders L = 27..32.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f32_d(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(float, 27)
        TCM_TILE_CASE(float, 28)
        TCM_TILE_CASE(float, 29)
        TCM_TILE_CASE(float, 30)
        TCM_TILE_CASE(float, 31)
        TCM_TILE_CASE(float, 32)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
