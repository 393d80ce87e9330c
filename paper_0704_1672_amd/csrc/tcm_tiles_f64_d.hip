// Moment-pass tile kernels, FP64 path, orders L = 27..32.
#include "tcm_device.h"

namespace tcm {

hipError_t launch_tiles_f64_d(int L, const DevPlan& P, int begin, int end, hipStream_t s)
{
    switch (L) {
        TCM_TILE_CASE(double, 27)
        TCM_TILE_CASE(double, 28)
        TCM_TILE_CASE(double, 29)
        TCM_TILE_CASE(double, 30)
        TCM_TILE_CASE(double, 31)
        TCM_TILE_CASE(double, 32)
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace tcm
