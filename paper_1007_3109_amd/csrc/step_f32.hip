// Step kernels for f32 population storage.
#include "lbrd_step_launch.h"

namespace lbrd {

hipError_t launch_step_f32(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    return launch_step_s<kF32>(sl, g, params, st);
}

hipError_t launch_stepT_f32(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    return launch_stepT_s<kF32>(sl, g, params, st);
}

}  // namespace lbrd
