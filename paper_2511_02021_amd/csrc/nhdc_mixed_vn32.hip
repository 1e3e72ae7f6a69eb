// nhdc_mixed_vn32.hip -- the mixed-precision form with the normal velocity
// (prognostic and predicted) stored in FP32, a variant of nhdc_mixed.hip:
// the same FP32 stencils and FP64 vertical solve, reference-state
// perturbations, fluxes and accumulators; the vn sum is formed in FP64 and
// rounded to FP32 where it is stored.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "nhdc_internal.h"

#pragma clang fp contract(fast)

namespace nhdc {
// a namespace of its own, so that profiles tell these kernels from the mixed
// form's (same names and template arguments)
namespace vn32 {
using VNT = float;  // the stored normal velocity
#include "nhdc_step.inc"
}  // namespace vn32

hipError_t launch_substep_mixed_vn32(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return vn32::substep<float>(L, sub, tm, st);
}

hipError_t launch_diffusion_mixed_vn32(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st) {
    return vn32::diffusion<float>(L, sub, tm, st);
}

hipError_t persistent_blocks_per_cu_mixed_vn32(const Launcher &L, int *blocks) {
    const void *k = nullptr;
    return vn32::persistent_props<float>(L, &k, blocks);
}

hipError_t launch_persistent_mixed_vn32(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                        hipStream_t st) {
    return vn32::persistent<float>(L, d_pm, sub, grid, st);
}

hipError_t launch_tracers_mixed_vn32(const Launcher &L, const Sub &sub, int phase, Timing *tm, hipStream_t st) {
    return vn32::tracers<float>(L, sub, phase, tm, st);
}
}  // namespace nhdc
