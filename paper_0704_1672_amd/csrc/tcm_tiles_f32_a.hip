// Moment-pass tile kernels, FP32 compensated path, orders L = 0..12.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f32_a(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(float, 0)
        TCM_TILE_CASE(float, 1)
        TCM_TILE_CASE(float, 2)
        TCM_TILE_CASE(float, 3)
        TCM_TILE_CASE(float, 4)
        TCM_TILE_CASE(float, 5)
        TCM_TILE_CASE(float, 6)
        TCM_TILE_CASE(float, 7)
        TCM_TILE_CASE(float, 8)
        TCM_TILE_CASE(float, 9)
        TCM_TILE_CASE(float, 10)
        TCM_TILE_CASE(float, 11)
        TCM_TILE_CASE(float, 12)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
