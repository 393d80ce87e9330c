// Moment-pass tile kernels, FP64 path, orders L = 0..12.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f64_a(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(double, 0)
        TCM_TILE_CASE(double, 1)
        TCM_TILE_CASE(double, 2)
        TCM_TILE_CASE(double, 3)
        TCM_TILE_CASE(double, 4)
        TCM_TILE_CASE(double, 5)
        TCM_TILE_CASE(double, 6)
        TCM_TILE_CASE(double, 7)
        TCM_TILE_CASE(double, 8)
        TCM_TILE_CASE(double, 9)
        TCM_TILE_CASE(double, 10)
        TCM_TILE_CASE(double, 11)
        TCM_TILE_CASE(double, 12)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
