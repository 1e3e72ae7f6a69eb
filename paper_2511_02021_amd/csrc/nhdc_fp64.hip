// nhdc_fp64.hip -- the FP64 form of the substep kernels.  Compiled without
// floating-point contraction: together with the operation order of
// nhdc_step.inc this makes every value bitwise equal to the plain FP64
// definition of the discretisation.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "nhdc_internal.h"

#pragma clang fp contract(off)

namespace nhdc {
using VNT = double;  // the stored normal velocity
#include "nhdc_step.inc"

hipError_t launch_substep_fp64(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return substep<double>(L, sub, tm, st);
}

hipError_t launch_diffusion_fp64(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return diffusion<double>(L, sub, tm, st);
}

hipError_t persistent_blocks_per_cu_fp64(const Launcher &L, int *blocks) {
    const void *k = nullptr;
    return persistent_props<double>(L, &k, blocks);
}

hipError_t launch_persistent_fp64(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                  hipStream_t st) {
    return persistent<double>(L, d_pm, sub, grid, st);
}

hipError_t launch_tracers_fp64(const Launcher &L, const Sub &sub, int phase, Timing *tm, hipStream_t st) {
    return tracers<double>(L, sub, phase, tm, st);
}
}  // namespace nhdc
