// nhdc_internal.h -- device-side data of one libnhdc context.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nhdc.h"

namespace nhdc {

// Connectivity and stencil coefficients (device pointers).  Pentagon pad
// slots point at a valid entity with a zero coefficient, so gathers need no
// branch.
struct Grid {
    int64_t nc = 0, ne = 0, nv = 0;
    int N = 0;
    double radius = 0, abar = 0;     // mean cell area 4 pi a^2 / nc
    int32_t *c_e = nullptr;          // [3][nc] cell -> edges
    int32_t *c_n = nullptr;          // [3][nc] neighbour across edge slot j
    int32_t *c_v = nullptr;          // [3][nc] vertex slot j (edge slot j joins vertex slots j, j+1)
    int32_t *e_c = nullptr;          // [2][ne] edge -> c1, c2
    int32_t *e_v = nullptr;          // [2][ne] edge -> v1, v2
    int32_t *v_e = nullptr;          // [6][nv] vertex ring edges (pad -> slot 0)
    int32_t *v_c = nullptr;          // [6][nv] vertex ring cells (pad -> slot 0)
    double *c_sl = nullptr;          // [3][nc] s(c,e_j) * l_ej
    double *c_area = nullptr;        // [nc] cell area
    double *c_x = nullptr;           // [3][nc] unit cell centre (radial direction)
    double *c_dv = nullptr;          // [9][nc] a*(x_ej - x_c), row j*3+d
    double *e_de = nullptr;          // [ne] dual length d_e
    double *e_le = nullptr;          // [ne] primal length l_e
    double *e_t = nullptr;           // [3][ne] edge tangent
    double *fe = nullptr;            // [ne] Coriolis parameter 2 Omega z_e
    double *v_sd = nullptr;          // [6][nv] sigma(v,e_j) * d_ej (0 on pad)
    double *v_m = nullptr;           // [6][nv] 1 on ring slots, 0 on pad
    double *v_val = nullptr;         // [nv] valence
    double *v_area = nullptr;        // [nv] dual area
    // vertical metrics
    double *zh = nullptr;            // [N+1][nc]
    double *gw = nullptr;            // [N+1][nc] interpolation weight (interior half levels)
    double *dref = nullptr;          // [N+1][nc] -g/(cpd theta_ref at half level)
    double *zhv = nullptr;           // [N+1][nv] vertex average of zh
    double *pi_ref = nullptr;        // [N][nc]
    double *theta_ref = nullptr;     // [N][nc]
};

struct State {
    double *vn = nullptr, *w = nullptr, *rho = nullptr, *pi = nullptr, *thv = nullptr,
           *pi_prev = nullptr;
    double *facc = nullptr, *wacc = nullptr;
};

// Work arrays of one substep.
struct Work {
    double *vt = nullptr;     // [N][ne] tangential velocity
    double *zeta = nullptr;   // [N][nv] vertex vorticity
    double *wv = nullptr;     // [N+1][nv] vertex average of w
    double *kc = nullptr;     // [N][nc] cell kinetic energy
    double *dvn = nullptr;    // [N][nc] divergence of vn (damping)
    double *wcc0 = nullptr, *tw0 = nullptr;  // [N+1][nc] of state n
    double *wcc1 = nullptr, *tw1 = nullptr;  // [N+1][nc] of the predicted state
    double *tvn0 = nullptr;   // [N][ne] vn tendency of state n
    double *gp = nullptr;     // [N][ne] terrain-corrected Exner gradient
    double *vns = nullptr;    // [N][ne] predicted vn
    double *flx = nullptr;    // [N][ne] edge mass flux
    double *hfl = nullptr;    // [N][ne] edge rho*theta_v flux
    double *ws = nullptr;     // [N+1][nc] predicted w
    double *rhos = nullptr;   // [N][nc] predicted rho
    double *thvs = nullptr;   // [N][nc] predicted theta_v
    double *cp = nullptr, *dp = nullptr;  // [N+1][nc] Thomas factors
    double *rh = nullptr, *ph = nullptr;  // [N][nc] explicit rho and Exner parts
    double *red = nullptr;    // reduction partials [2 * blocks + 2]
    int *flag = nullptr;      // finiteness flag
};

struct Params {
    double omega, grav, rd, cpd, p00, beta, wgt_corr, extrap, div_damp;
};

}  // namespace nhdc

namespace nhdc {
enum KernelId { K_VT_EDGE = 0, K_VERTEX, K_CELL_VT, K_EDGE_PRED, K_COLUMN_PRED, K_EDGE_CORR,
                K_COLUMN_CORR, K_NUM };
extern const char *const kKernelNames[K_NUM];

// Event timing of kernel launches within one nhdc_step call.
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pool: 2 per launch
    std::vector<int> ids;         // kernel id per launch of the current step
    double total_ms[K_NUM] = {0};
    int64_t launches[K_NUM] = {0};
};
}  // namespace nhdc

struct nhdc_ctx {
    int device = 0;
    int precision = NHDC_FP64;
    bool grid_ready = false, state_ready = false;
    nhdc::Grid g;
    nhdc::State s;
    nhdc::Work w;
    nhdc::Params p{};
    nhdc::Timing tm;
    std::vector<void *> allocs;
    std::string err;
};

namespace nhdc {
// kernels (nhdc_kernels.hip)
hipError_t launch_metrics(const Grid &g, const Params &p, hipStream_t st);
hipError_t launch_substep(nhdc_ctx *ctx, double dts, int nsub, bool first, hipStream_t st);
// timing helpers (no-ops unless ctx->tm.on)
hipError_t timing_begin(nhdc_ctx *ctx, int id, hipStream_t st);
hipError_t timing_end(nhdc_ctx *ctx, hipStream_t st);
hipError_t launch_diag(nhdc_ctx *ctx, double *out2, hipStream_t st);
hipError_t launch_finite(nhdc_ctx *ctx, int *flag, hipStream_t st);
hipError_t launch_init_prev(nhdc_ctx *ctx, hipStream_t st);
}  // namespace nhdc
