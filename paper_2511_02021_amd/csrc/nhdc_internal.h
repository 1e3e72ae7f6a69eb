// nhdc_internal.h -- device-side data of libnhdc contexts and batches.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nhdc.h"

namespace nhdc {

constexpr int BLOCK = 256;
// cell_vt's per-block tables: at most this many distinct edges, vertices and
// outside neighbours per block of BLOCK cells (a block of the bisection-curve
// numbering is one subtree of 256 triangles: 408, 153 and 48)
constexpr int CVT_E = 416, CVT_V = 160, CVT_X = 64;      // lanes per workgroup (4 wavefronts)
constexpr int MAX_INST = NHDC_MAX_INST;  // instances of one batched launch

// Stencil coefficients in one precision.  The FP64 form reads the double
// set; the mixed form's FP32 stencils read float copies of the same values.
// Fixed metric divisors are stored as their reciprocals (the IEEE quotient
// 1/x in FP64, as the operators scale by them).
template <class T>
struct Geo {
    T *c_sl = nullptr;    // [3][nc] s(c,e_j) * l_ej
    T *c_dv = nullptr;    // [9][nc] a*(x_ej - x_c), row j*3+d
    T *c_x = nullptr;     // [3][nc] unit cell centre (radial direction)
    T *c_area = nullptr;  // [nc] cell area (mass sums)
    T *c_ia = nullptr;    // [nc] 1 / cell area
    T *e_ide = nullptr;   // [ne] 1 / dual length d_e
    T *e_ile = nullptr;   // [ne] 1 / primal length l_e
    T *e_t = nullptr;     // [3][ne] edge tangent
    T *fe = nullptr;      // [ne] Coriolis parameter 2 Omega z_e
    T *v_sd = nullptr;    // [6][nv] sigma(v,e_j) * d_ej (0 on the pentagon pad)
    T *v_m = nullptr;     // [6][nv] 1 on ring slots, 0 on the pad
    T *v_ival = nullptr;  // [nv] 1 / valence
    T *v_ia = nullptr;    // [nv] 1 / dual area
};

struct Grid {
    int64_t nc = 0, ne = 0, nv = 0;
    int N = 0;
    double radius = 0, abar = 0;  // mean cell area 4 pi a^2 / nc
    int32_t *c_e = nullptr;       // [3][nc] cell -> edges
    int32_t *c_n = nullptr;       // [3][nc] neighbour across edge slot j
    int32_t *c_v = nullptr;       // [3][nc] vertex slot j (edge slot j joins vertex slots j, j+1)
    int32_t *e_c = nullptr;       // [2][ne] edge -> c1, c2
    int32_t *e_v = nullptr;       // [2][ne] edge -> v1, v2
    int32_t *v_e = nullptr;       // [6][nv] vertex ring edges (pad -> slot 0)
    int32_t *v_c = nullptr;       // [6][nv] vertex ring cells (pad -> slot 0)
    int32_t *c_ns = nullptr;      // [3][nc] slot of the shared edge in the neighbour across slot j
    // cells shared by a block of BLOCK consecutive edges: the block's distinct
    // cells in ascending order (padded with its first), their count, and each
    // edge's c1 and c2 as positions in its block's list
    int32_t *eb_cells = nullptr;  // [ceil(ne / BLOCK)][2 BLOCK]
    int32_t *eb_n = nullptr;      // [ceil(ne / BLOCK)]
    int32_t *e_loc = nullptr;     // [2][ne]
    int32_t eb_max = 0;           // the most distinct cells of any block
    // the same for blocks of BLOCK consecutive cells (cell_vt), when every
    // block fits the CVT_* sizes (cvt_ok): distinct edges, vertices and
    // neighbours outside the block (ascending, padded with the first), their
    // three counts per block [3][nblk], and each cell's slots as positions:
    // edges and vertices in the block's lists, neighbours as the cell's
    // position in the block or BLOCK + position in the outside list
    int32_t cvt_ok = 0;
    int32_t *cb_e = nullptr, *cb_v = nullptr, *cb_x = nullptr, *cb_n = nullptr;
    int32_t *c_el = nullptr, *c_vl = nullptr, *c_nl = nullptr;  // [3][nc]
    Geo<double> gd;
    Geo<float> gf;
    // second-order upwind option (FP64; allocated only with the option)
    double *e_frac = nullptr;     // [ne] edge midpoint's position on the dual arc c1 -> c2
    double *e_n = nullptr;        // [3][ne] edge normal
    double *e_d1 = nullptr;       // [3][ne] a (x_e - x_c1)
    double *e_d2 = nullptr;       // [3][ne] a (x_e - x_c2)
    // sponge option: Rayleigh damping rate of w per half level [N+1] (or null)
    double *w_damp = nullptr;
    double *zh = nullptr;         // [N+1][nc] half-level heights
    // leading half levels (from the lid down) at which every cell's zh, and
    // every vertex's zhv, has the same bits: there a neighbour's height is the
    // level's first entry, read without a gather
    int32_t flat_c = 0, flat_v = 0;
    int32_t flat_r = 0;           // the same for pi_ref and theta_ref (full levels)
    double *zhv = nullptr;        // [N+1][nv] vertex average of zh
    double *pi_ref = nullptr;     // [N][nc]
    double *theta_ref = nullptr;  // [N][nc]
};

template <class T>
__host__ __device__ inline const Geo<T> &geo(const Grid &g);
template <>
__host__ __device__ inline const Geo<double> &geo<double>(const Grid &g) { return g.gd; }
template <>
__host__ __device__ inline const Geo<float> &geo<float>(const Grid &g) { return g.gf; }

// Prognostic state (FP64 in every form) and the FP64 mass-flux accumulators.
// px is derived: the extrapolated Exner perturbation (1+eps)(pi - pi_ref) -
// eps pi_prev that the next predictor uses, kept current by every call that
// changes the state (the corrector's column writes it for the next substep).
// pi_prev itself is only read back by callers, so the corrector stores it on
// the last substep of a step.
struct State {
    double *vn = nullptr, *w = nullptr, *rho = nullptr, *pi = nullptr, *thv = nullptr,
           *pi_prev = nullptr;
    double *facc = nullptr, *wacc = nullptr;
    double *px = nullptr;  // [N][nc]
};

// Work arrays of one substep.  Tendency-side arrays have the stencil
// precision RT; predicted state, fluxes and column scratch are FP64.
template <class RT>
struct Work {
    RT *vt = nullptr;     // [N][ne] tangential velocity
    RT *zeta = nullptr;   // [N][nv] vertex vorticity
    RT *wv = nullptr;     // [N+1][nv] vertex average of w
    RT *kc = nullptr;     // [N][nc] cell kinetic energy
    RT *dvn = nullptr;    // [N][nc] divergence of vn (damping)
    RT *wcc0 = nullptr, *tw0 = nullptr;  // [N+1][nc] of state n
    RT *wcc1 = nullptr, *tw1 = nullptr;  // [N+1][nc] of the predicted state
    RT *tvn0 = nullptr;   // [N][ne] vn tendency of state n
    double *vns = nullptr;    // [N][ne] predicted vn
    double *fh = nullptr;     // [N][ne][2] edge mass flux and rho*theta_v flux, paired
    double *ws = nullptr;     // [N+1][nc] predicted w
    double *rhos = nullptr;   // [N][nc] predicted rho
    double *thvs = nullptr;   // [N][nc] predicted theta_v
    double *cd = nullptr;     // [N+1][nc][2] Thomas factors c', d', paired
    double *rp = nullptr;     // [N][nc][2] explicit rho and Exner parts, paired
    double *gq = nullptr;  // [N][nc][6] cell gradients of rho, then theta_v (upwind)
    RT *dd4 = nullptr;     // [N][nc] D(G(D(vn*))) (fourth-order divergence damping)
    RT *kh = nullptr;      // [N][nc] Smagorinsky coefficient of the cell (diffusion)
};

// Tracers (option): mixing ratios carried by the step's averaged mass fluxes,
// FP64 in every form, and their scratch.
struct Tracers {
    int32_t nt = 0;
    double *q = nullptr;     // [nt][N][nc] mixing ratios
    double *rec = nullptr;   // [nt][3][N][nc] linear reconstruction toward edge slot j
    double *qs = nullptr;    // [nt][N][nc] after the horizontal update
    double *rs = nullptr;    // [N][nc] density after the horizontal update
    double *rho0 = nullptr;  // [N][nc] density at the start of the step
};

struct Params {
    double omega, grav, rd, cpd, p00, beta, wgt_corr, extrap, div_damp;
    int32_t upwind;    // 1: second-order upwind edge values of rho and theta_v in the fluxes
    double div_damp4;  // fourth-order divergence damping coefficient (0: off)
    double smag;       // Smagorinsky constant of the diffusion of vn (0: off)
};

// Everything one kernel needs about one instance (lives in device memory).
template <class RT>
struct Inst {
    Grid g;
    State s;
    Work<RT> w;
    Params p;
    Tracers tr;
};

// Entity kinds of a launch, each with its own block map.
enum Kind { KIND_EDGE = 0, KIND_CELL, KIND_VERT, KIND_COLUMN, KIND_NUM };

// Block map of one launch over a batch: instance i owns global tiles
// [off[i], off[i+1]); within it, tile t covers entity block t % nbe[i] and
// levels [lt[i] * (t / nbe[i]), ...).
struct Map {
    int32_t n = 0;
    int32_t off[MAX_INST + 1] = {0};
    int32_t nbe[MAX_INST] = {0};
    int32_t lt[MAX_INST] = {0};
};

// Block maps and tile counts of every kind, in device memory for the
// persistent launch.
struct PMaps {
    Map maps[KIND_NUM];
    int64_t nblocks[KIND_NUM];
};

// Per-launch scalars of one substep.
struct Sub {
    double dt[MAX_INST];
    int32_t nsub, first, last;  // substeps per step; first / last substep of the step
};

// Level-tile sizes (levels per lane) of the marching kernels (0 = whole
// column), and the block sizes of the kernels that take several (the column
// and vertex kernels: 64, 128 or 256 lanes; the others keep BLOCK, which
// their per-block tables and LDS arrays are built for).
// col_waves caps the waves per SIMD of the column kernel (0: as many as its
// registers allow, 4) by reserving LDS per block: fewer columns in flight at
// once keep more of their scratch round trip in the caches (3 measured best).
// The defaults are the shapes the autotuner picks for the R2B6x90 and
// R2B8x90 workloads (the vertex kernel in blocks of 64: 1 % faster at R2B6,
// the same at R2B8).
// col_mode selects the column build: 0 one lane per column, marching down
// and up the whole column (the streaming build); 1 the level-parallel build,
// the levels of a column shared among lanes and the Thomas factors in LDS
// (k_column_stg).  Both give the same results to the bit.
struct Tune {
    int lt_edge = 0, lt_cell = 0, lt_vert = 0;
    int blk_col = BLOCK, blk_vert = 64;
    int col_waves = 3;
    int col_mode = 0;
};
inline bool same_tune(const Tune &a, const Tune &b) {
    return a.lt_edge == b.lt_edge && a.lt_cell == b.lt_cell && a.lt_vert == b.lt_vert &&
           a.blk_col == b.blk_col && a.blk_vert == b.blk_vert && a.col_waves == b.col_waves &&
           a.col_mode == b.col_mode;
}
inline bool valid_col_mode(int m) { return m == 0 || m == 1; }
// The level-parallel column: its LDS per block for up to nmax levels (six
// arrays of nmax + 1 rows of C + 1 doubles), and its columns per block: 16
// (a wavefront's 16-column rows then read whole 128-byte lines), or 8 or 4
// where the arrays would exceed the device's LDS per block
inline unsigned stg_lds(int width, int nmax) { return unsigned(6 * (nmax + 1) * (width + 1) * 8); }
inline int stg_width(int nmax, int max_lds) {
    for (int w = 16; w > 4; w /= 2)
        if (stg_lds(w, nmax) <= unsigned(max_lds)) return w;
    return 4;
}
inline bool valid_block(int b) { return b == 64 || b == 128 || b == 256; }
inline bool valid_waves(int w) { return w == 0 || w == 2 || w == 3; }
// LDS per block that lets a CU (160 KB of LDS, 4 SIMDs of 64-lane waves)
// hold `waves` waves per SIMD of `block`-lane blocks but not one block more
inline unsigned occupancy_lds(int waves, int block) {
    if (waves <= 0) return 0;
    const int blocks = waves * 4 * 64 / block;
    return unsigned(163840 / (blocks + 1) + 256);
}

enum KernelId { K_VT_EDGE = 0, K_VERTEX, K_CELL_VT, K_EDGE_PRED, K_COLUMN_PRED, K_EDGE_CORR,
                K_COLUMN_CORR, K_CELL_GRAD, K_DIV4, K_SMAG_CELL, K_SMAG_EDGE, K_TR_SAVE,
                K_TR_RECON, K_TR_HORIZ, K_TR_VERT, K_NUM };
extern const char *const kKernelNames[K_NUM];

// Event timing of kernel launches within one step call.
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pool: 2 per launch
    std::vector<int> ids;         // kernel id per launch of the current step
    double total_ms[K_NUM] = {0};
    int64_t launches[K_NUM] = {0};
};

// Device memory source of a context: the caller's callbacks
// (nhdc_set_allocator), or hipMalloc / hipFree when none are set.
struct Allocator {
    void *(*alloc)(size_t bytes, void *user) = nullptr;
    void (*free_)(void *ptr, void *user) = nullptr;
    void *user = nullptr;
};
// bytes of device memory from `a` (nullptr on failure), and their release
void *dev_alloc(const Allocator &a, size_t bytes);
void dev_free(const Allocator &a, void *p);

// One set of instances advanced together (a context is a batch of one).
struct Launcher {
    Allocator al;                  // where d_insts (and autotuning snapshots) come from
    int precision = NHDC_FP64;
    int n = 0;
    void *d_insts = nullptr;       // Inst<double>[n] or Inst<float>[n] in device memory
    bool upwind = false;           // some instance uses the second-order upwind option
    bool div4 = false;             // some instance uses fourth-order divergence damping
    bool smag = false;             // some instance uses the Smagorinsky diffusion
    bool sponge = false;           // some instance has a Rayleigh sponge on w
    bool tracers = false;          // some instance carries tracers
    bool vt_two = false;           // some edge block has more distinct cells than lanes
    bool cvt_lds = false;          // every instance has cell_vt's block tables
    Map maps[KIND_NUM];
    int64_t nblocks[KIND_NUM] = {0};
    int block[KIND_NUM] = {BLOCK, BLOCK, BLOCK, BLOCK};  // lanes per block of each kind's launches
    unsigned dyn_lds[KIND_NUM] = {0, 0, 0, 0};           // LDS per block (occupancy cap, or the staged column's arrays)
    int col_width = 0;             // columns per block of the level-parallel column (0: streaming build)
    Map trmap;                     // the tracers' column march: whole columns, blocks of BLOCK lanes
    int64_t trblocks = 0;
};

// kernels (nhdc_fp64.hip / nhdc_mixed.hip / nhdc_mixed_vn32.hip)
hipError_t launch_substep_fp64(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
hipError_t launch_substep_mixed(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
hipError_t launch_substep_mixed_vn32(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
hipError_t launch_diffusion_mixed_vn32(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
hipError_t launch_tracers_mixed_vn32(const Launcher &L, const Sub &sub, int phase, Timing *tm,
                                     hipStream_t st);
// the diffusion after the substeps of a step (sub.dt: the step's dt per instance)
hipError_t launch_diffusion_fp64(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
hipError_t launch_diffusion_mixed(const Launcher &L, const Sub &sub, Timing *tm, hipStream_t st);
// tracers: phase 0 keeps the density at the start of a step, phase 1
// transports over the step (sub.dt: the step's dt per instance)
hipError_t launch_tracers_fp64(const Launcher &L, const Sub &sub, int phase, Timing *tm, hipStream_t st);
hipError_t launch_tracers_mixed(const Launcher &L, const Sub &sub, int phase, Timing *tm, hipStream_t st);
// the persistent form of a batch step's substeps: one cooperative launch of
// `grid` blocks (sub.nsub substeps); and how many of its blocks a CU holds
hipError_t launch_persistent_fp64(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                  hipStream_t st);
hipError_t launch_persistent_mixed(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                   hipStream_t st);
hipError_t launch_persistent_mixed_vn32(const Launcher &L, const PMaps *d_pm, const Sub &sub, int grid,
                                        hipStream_t st);
hipError_t persistent_blocks_per_cu_fp64(const Launcher &L, int *blocks);
hipError_t persistent_blocks_per_cu_mixed(const Launcher &L, int *blocks);
hipError_t persistent_blocks_per_cu_mixed_vn32(const Launcher &L, int *blocks);
// The launches of one precision form.
struct FormOps {
    hipError_t (*substep)(const Launcher &, const Sub &, Timing *, hipStream_t);
    hipError_t (*diffusion)(const Launcher &, const Sub &, Timing *, hipStream_t);
    hipError_t (*tracers)(const Launcher &, const Sub &, int, Timing *, hipStream_t);
    hipError_t (*persistent)(const Launcher &, const PMaps *, const Sub &, int, hipStream_t);
    hipError_t (*persistent_blocks)(const Launcher &, int *);
};
const FormOps &form_ops(int precision);
// the stencils of a precision run in FP32 (the mixed forms)
inline bool fp32_stencils(int precision) { return precision != NHDC_FP64; }
// bytes of one stored normal velocity (FP32 in the mixed form's FP32-vn variant)
inline int vn_bytes(int precision) { return precision == NHDC_MIXED_VN32 ? 4 : 8; }
// set-up and diagnostics (nhdc_util.hip)
hipError_t launch_metrics(const Grid &g, hipStream_t st);
// out[i] |= 1 where row i of the [nlev][n] array a has an entry whose bits
// differ from its first entry's
hipError_t launch_level_nonflat(const double *a, int64_t n, int nlev, int32_t *out, hipStream_t st);
hipError_t launch_to_float(const double *src, float *dst, int64_t n, hipStream_t st);
hipError_t launch_to_double(const float *src, double *dst, int64_t n, hipStream_t st);
hipError_t launch_diag(const Grid &g, const State &s, double *part, double *out2, hipStream_t st);
hipError_t launch_finite(const Grid &g, const State &s, int vn_size, int *flag, hipStream_t st);
// release a context's device memory and the context (nhdc_destroy, or the
// last batch holding a context whose destroy was deferred)
void free_context(nhdc_ctx *ctx);
// message of the calling thread's last failed context-free call
const char *context_free_error();
hipError_t launch_init_prev(const Grid &g, const State &s, hipStream_t st);
hipError_t launch_exner_x(const Grid &g, const State &s, double eps, hipStream_t st);
// timing helpers (nhdc_runtime.hip); no-ops when tm is null or off
hipError_t timing_begin(Timing *tm, int id, hipStream_t st);
hipError_t timing_end(Timing *tm, hipStream_t st);
// block map of one kind over a set of grids, with that kind's block size
// (entities: the entities per block when > 0, else the kind's block size)
void build_map(Map &m, int64_t &nblocks, Kind kind, const Grid *const *grids, int n,
               const Tune &t, int entities = 0);
// LDS bytes one block may use on a device (cached per device)
int device_max_lds(int device);
int kind_block(Kind kind, const Tune &t);

}  // namespace nhdc

struct nhdc_ctx {
    int device = 0;
    int precision = NHDC_FP64;
    bool grid_ready = false, state_ready = false;
    nhdc::Grid g;
    nhdc::State s;
    nhdc::Work<double> wd;
    nhdc::Work<float> wf;
    nhdc::Params p{};
    nhdc::Tracers tr;
    std::vector<void *> tr_allocs;  // tracer arrays (freed when the tracers are replaced)
    int in_batches = 0;             // live batches holding this context's descriptor
    bool destroy_pending = false;   // nhdc_destroy came while batched: freed by the last batch
    nhdc::Allocator al;             // device memory source (nhdc_set_allocator)
    // mixed forms: one device allocation holding the grid, state and work
    // arrays of the context (sized at upload), from which they are carved in
    // turn at 2 MiB boundaries: one contiguous range instead of some sixty
    // separate allocations measured 5-7 % faster steps at R2B8x90 (the FP64
    // form measured the same or slower and keeps separate allocations)
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    nhdc::Tune tune;
    nhdc::Launcher L;
    nhdc::Timing tm;
    double *red = nullptr;   // reduction partials [2 * blocks + 2]
    int *flag = nullptr;     // finiteness flag
    std::vector<void *> allocs;
    std::string err;
};
