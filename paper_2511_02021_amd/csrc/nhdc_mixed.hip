// nhdc_mixed.hip -- the mixed-precision form of the substep kernels:
// horizontal stencils and velocity tendencies in FP32 (with fused
// multiply-add); the vertically implicit solve, the reference-state
// perturbations, the edge fluxes, their divergences and the mass-flux
// accumulators in FP64, as is the prognostic state.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "nhdc_internal.h"

#pragma clang fp contract(fast)

namespace nhdc {
using VNT = double;  // the stored normal velocity
#include "nhdc_step.inc"

hipError_t launch_substep_mixed(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return substep<float>(L, sub, tm, st);
}

hipError_t launch_diffusion_mixed(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return diffusion<float>(L, sub, tm, st);
}

hipError_t persistent_blocks_per_cu_mixed(const Launcher &L, int *blocks) {
    const void *k = nullptr;
    return persistent_props<float>(L, &k, blocks);
}

hipError_t launch_persistent_mixed(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                  hipStream_t st) {
    return persistent<float>(L, d_pm, sub, grid, st);
}

hipError_t launch_tracers_mixed(const Launcher &L, const Sub &sub, int phase, Timing *tm, hipStream_t st) {
    return tracers<float>(L, sub, phase, tm, st);
}
}  // namespace nhdc
