// Step kernels for bf16 population storage.
#include "lbrd_step_launch.h"

namespace lbrd {

hipError_t launch_step_bf16(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    return launch_step_s<kBF16>(sl, g, params, st);
}

hipError_t launch_stepT_bf16(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    return launch_stepT_s<kBF16>(sl, g, params, st);
}

}  // namespace lbrd
