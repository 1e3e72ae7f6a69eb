/*
 * nhdc.h -- C-ABI of the MI355X (gfx950) nonhydrostatic dynamical-core
 * substep library libnhdc.so.
 *
 * The library advances the atmosphere's dynamical core on the icosahedral
 * triangular C grid (paper Sec. 2: nonhydrostatic formulation on the
 * icosahedral-triangular C grid with a terrain-following hybrid height
 * coordinate; Table 2: normal velocity on edges, 90 levels; Sec. 3.2: the
 * dynamical core is memory-bandwidth bound and dominated by indirect
 * neighbour lookups).  The boundary follows the problem statement: upload a
 * grid with its connectivity and vertical coordinate, initialise a state, then
 * step(dt, nsubsteps).  Every step of the path runs in HIP kernels on the GPU;
 * the state stays resident in device memory between calls (Sec. 3.1: data
 * stay on the GPU for the whole run).
 *
 * One substep (length dt/nsubsteps) is: velocity tendencies of the current
 * state; extrapolated Exner perturbation and its terrain-corrected normal
 * gradient; predicted normal velocity, edge mass and rho*theta_v fluxes and
 * their divergences; a vertically implicit tridiagonal solve per column for
 * w and Exner pressure (with rho and theta_v updates); velocity tendencies of
 * the predicted state; corrected normal velocity with averaged tendencies and
 * divergence damping; fluxes; the implicit column solve again about the old
 * state with interface values averaged between old and predicted; FP64
 * accumulation of the mass fluxes.
 *
 * Options (nhdc_params, nhdc_vertical, nhdc_set_tracers; all off by default):
 * second-order upwind edge values of rho and theta_v in the fluxes; fourth-
 * order divergence damping; a Rayleigh sponge on w in the column solves;
 * Smagorinsky diffusion of vn once per step; and tracers carried by the
 * step's averaged mass fluxes (Sec. 1 counts water vapour, carbon dioxide and
 * ozone among the atmosphere's prognostic quantities; Table 2).
 *
 * Conventions
 *  - Return values: NHDC_OK (0) or a negative NHDC_E* code; nothing throws or
 *    aborts across the ABI.  nhdc_last_error(ctx) gives the message of the
 *    last failure of that context.
 *  - Arrays: FP64 unless stated, level-major [k][i] (entity index fastest).
 *    Full levels k = 0..N-1 top to bottom; half levels i = 0..N, half level i
 *    is the top interface of full level i, i = N the ground.  Connectivity is
 *    int32 slot-major [slot][i], -1 padded (see nhgrid.h for the conventions).
 *  - Ownership: the caller owns every array it passes; upload and init copy.
 *    The context owns its device memory until nhdc_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  nhdc_step only enqueues work; the caller synchronises.
 *  - Numbering: arrays are used in the order given (the library never
 *    renumbers); a space-filling-curve order (nhgrid_reorder) makes the
 *    indirect gathers coalesce.
 *  - Threading: one context is used by one host thread at a time; distinct
 *    contexts are independent.
 */
#ifndef NHDC_H
#define NHDC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NHDC_OK = 0,
    NHDC_EINVAL = -1,    /* bad argument: NULL pointer, dt <= 0 or not finite, nsub < 1, size mismatch */
    NHDC_ENOMEM = -2,    /* device or host allocation failed */
    NHDC_EHIP = -3,      /* a HIP runtime call failed (message has hipGetErrorString) */
    NHDC_EGRID = -4,     /* grid or vertical coordinate failed validation */
    NHDC_ESTATE = -5,    /* call out of order (e.g. step before init) */
    NHDC_EUNSTABLE = -6, /* non-finite value found by nhdc_check_finite */
    NHDC_ETOOBIG = -7    /* input larger than a fixed maximum (nhdc_diag_noalloc) */
};

/* Precision forms: NHDC_FP64 (every operation FP64); NHDC_MIXED (FP32
 * horizontal stencils and tendencies, FP64 state, vertical solve,
 * reference-state perturbations and mass fluxes); NHDC_MIXED_VN32 (as
 * NHDC_MIXED with the normal velocity, prognostic and predicted, stored in
 * FP32: its FP64 sum is rounded where it is stored; the boundary still takes
 * and gives FP64 vn). */
enum { NHDC_FP64 = 0, NHDC_MIXED = 1, NHDC_MIXED_VN32 = 2 };

typedef struct nhdc_ctx nhdc_ctx;

/* Grid: host arrays, same layout as nhgrid_view (nhgrid.h). */
typedef struct nhdc_grid {
    int64_t n_cells, n_edges, n_verts;
    double radius;
    const int32_t *cell_edges;   /* [3][n_cells] */
    const int8_t *cell_sign;     /* [3][n_cells] s(c,e): +1 if the edge normal points out of c */
    const int32_t *edge_cells;   /* [2][n_edges] c1, c2 (normal points from c1 to c2) */
    const int32_t *edge_verts;   /* [2][n_edges] v1, v2 (tangent points from v1 to v2) */
    const int32_t *vert_edges;   /* [6][n_verts] counter-clockwise ring, -1 pad */
    const int32_t *vert_cells;   /* [6][n_verts] ring cell j between ring edges j and j+1 */
    const int8_t *vert_sign;     /* [6][n_verts] +1 if the vertex is v2 of the edge */
    const int32_t *vert_valence; /* [n_verts] 5 or 6 */
    const double *cell_x;        /* [3][n_cells] unit circumcentres */
    const double *cell_area;     /* [n_cells] m^2 */
    const double *edge_x;        /* [3][n_edges] unit edge midpoints */
    const double *edge_tangent;  /* [3][n_edges] */
    const double *edge_length;   /* [n_edges] primal length [m] */
    const double *dual_length;   /* [n_edges] distance between the two circumcentres [m] */
    const double *vert_area;     /* [n_verts] dual area [m^2] */
    /* read only with the upwind option (may be NULL otherwise): */
    const double *edge_normal;   /* [3][n_edges] unit normal n_e (from c1 towards c2) */
    const double *dual_frac;     /* [n_edges] position of the edge midpoint on the dual
                                    arc c1 -> c2, as a fraction of its length (0..1) */
} nhdc_grid;

/* Vertical coordinate and reference profile of one column set (host arrays). */
typedef struct nhdc_vertical {
    int32_t n_lev;             /* N, 2 <= N <= NHDC_MAX_LEV */
    const double *zh;          /* [N+1][n_cells] half-level heights, strictly decreasing in i */
    const double *pi_ref;      /* [N][n_cells] reference Exner pressure at full levels */
    const double *theta_ref;   /* [N][n_cells] reference potential temperature at full levels */
    const double *w_damp;      /* [N+1] Rayleigh damping rate of w per half level [1/s], >= 0,
                                  or NULL for no sponge.  Each column solve (predictor and
                                  corrector) multiplies its solved w at interior half level i by
                                  1/(1 + dt_s w_damp[i]) before the mass, Exner and theta_v
                                  updates use it, so the sponge keeps the flux form. */
} nhdc_vertical;

#define NHDC_MAX_LEV 256

typedef struct nhdc_params {
    double omega;     /* planetary rotation [1/s] (Coriolis 2*omega*z at edge midpoints) */
    double grav, rd, cpd, p00;
    double beta;      /* implicit weight of the vertical solve (0.5..1) */
    double wgt_corr;  /* weight of the predicted-state tendency in the corrector */
    double extrap;    /* extrapolation factor of the Exner perturbation */
    double div_damp;  /* second-order divergence damping coefficient (times mean cell area) */
    int32_t upwind;   /* edge values of rho and theta_v in the mass and theta fluxes:
                         0 the centred average of the two cells; 1 second-order upwind:
                         the upwind cell's value plus its horizontal gradient (Green-Gauss,
                         edge values interpolated along the dual arc to the edge midpoint)
                         dotted with the displacement to the midpoint of the edge
                         midpoint's back trajectory over the substep, dt/2 (vn n + vt t) */
    double div_damp4; /* fourth-order divergence damping coefficient c4 >= 0 (0: off): the
                         corrector adds -c4 Abar^2 G(D(G(D(vn*)))) to vn, Abar the mean cell
                         area, G the normal gradient and D the divergence of the C-grid */
    double smag;      /* Smagorinsky constant c_s >= 0 (0: off): after the substeps of each
                         step, vn += dt K_e (G(D(vn)) - T(Z(vn))) with K_e the mean of its two
                         cells' c_s^2 A_c |Def|, capped at Abar/(25 dt); |Def| is the
                         tension-shear magnitude of the cell's Green-Gauss velocity-gradient
                         tensor of vn n + vt t on the tangent plane.  Needs edge_normal. */
} nhdc_params;

/* Prognostic state; pointers are host or device memory per `on_device`.
 * vn [N][n_edges], w [N+1][n_cells], rho, pi (Exner), theta_v, pi_prev [N][n_cells].
 * pi_prev is the Exner perturbation (pi - pi_ref) of the previous substep; on
 * init it may be NULL, meaning pi - pi_ref (the first extrapolation is then
 * the identity). */
typedef struct nhdc_state_view {
    double *vn, *w, *rho, *pi, *theta_v, *pi_prev;
    int32_t on_device;
} nhdc_state_view;

/* Create a context on HIP device `device` with precision NHDC_FP64 (every
 * operation in FP64, the precision the paper's memory accounting assumes,
 * Sec. 1), NHDC_MIXED (horizontal stencils and tendencies in FP32; vertical
 * solve, reference-state perturbations and mass fluxes FP64; the paper has no
 * reduced-precision form) or NHDC_MIXED_VN32.  No device memory is taken yet.
 * Errors: EINVAL for out NULL or an unknown precision, EHIP for a device that
 * does not exist, ENOMEM when the host context cannot be made. */
int nhdc_create(nhdc_ctx **out, int precision, int device);

/* Device memory source of the context (the paper keeps the model's data
 * resident on the GPU for the whole run, Sec. 3.1, so a caller that manages
 * device memory itself, e.g. PyTorch's caching allocator, can own it).  Every
 * device allocation the context makes from here on (grid, state, work
 * arrays, tracers, its launch descriptors, autotuning snapshots; also the
 * descriptors of a batch whose first instance it is) calls
 * alloc(bytes, user), which returns device memory of the context's device
 * (NULL on failure: the calling entry point then returns ENOMEM), and every
 * release calls free_(ptr, user) after the device has finished all work.
 * The callbacks and `user` must stay valid until nhdc_destroy has returned.
 * Both NULL restores hipMalloc / hipFree (the default).  Must be called
 * before nhdc_upload_grid (ESTATE afterwards); EINVAL if only one callback
 * is given. */
int nhdc_set_allocator(nhdc_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                       void (*free_)(void *ptr, void *user), void *user);

/* The grid upload of the problem statement: the icosahedral-triangular C
 * grid with its dual (Sec. 2; triangles, their hexagon/pentagon dual and the
 * integer index lookups between them, Sec. 3.2), the terrain-following
 * height coordinate (Sec. 2) and the reference profile.  Host arrays, copied;
 * the caller keeps ownership.
 * Copy and validate the grid (index ranges, edge-cell consistency, signs,
 * positive lengths and areas) and the vertical coordinate; derive device
 * metrics and stencil coefficients.  It also records how many half levels
 * from the lid carry the same height bits in every column (the flat top of a
 * terrain-following coordinate), and how many full levels the same reference
 * profile; the kernels read those levels from one entry, with unchanged
 * results.  It lists, per block of 256 edges and per block of 256 cells, the
 * distinct cells (edges, vertices, outside neighbours) the block's lanes share
 * through LDS.  May be called once per context. */
int nhdc_upload_grid(nhdc_ctx *ctx, const nhdc_grid *grid, const nhdc_vertical *vert,
                     const nhdc_params *params);

/* State initialisation (the paper starts from an interpolated initial
 * state, Sec. 4.1; here any state the caller gives).  Copy the initial state
 * (host or device memory per state->on_device; the caller keeps ownership);
 * zeroes the flux accumulators.  The state then stays resident on the device
 * between steps (Sec. 3.1).  Errors: EINVAL for a NULL field, ESTATE before
 * nhdc_upload_grid, EHIP when a copy fails.  Host copies are complete when
 * it returns; device copies are ordered on `stream`. */
int nhdc_init_state(nhdc_ctx *ctx, const nhdc_state_view *state, void *stream);

/* step(dt, nsubsteps) of the problem statement: the nonhydrostatic
 * dynamical core (Sec. 2) on the device, memory-bandwidth bound (Sec. 3.2).
 * Enqueue nsubsteps substeps of dt/nsubsteps.  The mass-flux accumulators are
 * restarted at entry and hold the average over these substeps afterwards.
 * With the options set, the step also runs the diffusion of vn over dt after
 * the substeps, and then the tracer transport with the averaged fluxes.
 * Errors: EINVAL for dt <= 0 or not finite and nsubsteps < 1, ESTATE before
 * a state is initialised, EHIP when a launch fails. */
int nhdc_step(nhdc_ctx *ctx, double dt, int nsubsteps, void *stream);

/* Copy the state into caller buffers (host or device per dst->on_device;
 * NULL members are skipped; the caller owns them).  Host copies are complete
 * when this returns.  The layout is that of nhdc_state_view.  Errors: EINVAL
 * for dst NULL, ESTATE before a state is initialised, EHIP when a copy
 * fails. */
int nhdc_get_state(nhdc_ctx *ctx, const nhdc_state_view *dst, void *stream);

/* Tracers (option), up to NHDC_MAX_TRACERS mixing ratios q [n][N][n_cells]
 * (host or device memory per on_device), copied; n = 0 removes them.  Each
 * step transports them after its substeps with the step's averaged FP64 mass
 * fluxes (the paper carries water vapour, carbon dioxide and ozone this way),
 * in FP64 in both precision forms:
 *   horizontal, flux form: the edge flux is Facc times the upwind cell's
 *     linear reconstruction q_c + grad(q)_c . a (x_e - x_c), upwind = c1 when
 *     Facc >= 0, grad the Green-Gauss gradient in difference form
 *     (1/A) sum_j s l w_j (q_nb - q_c) n_j (w_j the fraction of the dual arc
 *     from the cell to the edge midpoint), radial part removed; the density
 *     takes the divergence of the same fluxes from its value at the start of
 *     the step;
 *   vertical, piecewise parabolic: interface values from the cubic through
 *     four cell means on the stretched levels (linear next to the lid and the
 *     ground), the flux Wacc times the parabola's mean over the swept
 *     fraction |Wacc| dt / (rho dz) of the upwind cell (capped at 1).
 * A constant tracer stays exactly constant and tracer mass is conserved.
 * Needs a grid uploaded with edge_normal and dual_frac.  Calls the stream's
 * and the device's pending work to finish first.  Refused (ESTATE) while the
 * context is part of a live batch: set tracers before making the batch. */
#define NHDC_MAX_TRACERS 16
int nhdc_set_tracers(nhdc_ctx *ctx, int n_tracers, const double *q, int on_device, void *stream);
/* Copy the tracers out ([n][N][n_cells]); nothing when there are none. */
int nhdc_get_tracers(nhdc_ctx *ctx, double *q, int on_device, void *stream);
/* Number of tracers of the context. */
int nhdc_n_tracers(const nhdc_ctx *ctx);

/* Substep-averaged FP64 mass fluxes of the last step, which transport the
 * atmosphere's tracers (water vapour, carbon dioxide and ozone, Sec. 1):
 * edge fluxes rho*vn*dz [N][n_edges] (kg/m/s per unit edge length and layer)
 * and vertical fluxes at half levels [N+1][n_cells] (kg/m^2/s), into caller
 * buffers (host or device per on_device; NULL skips one).  Errors: ESTATE
 * before a state is initialised, EHIP when a copy fails. */
int nhdc_get_mass_flux(nhdc_ctx *ctx, double *facc, double *wacc, int on_device, void *stream);

/* Global dry mass sum A_c dz rho and sum A_c dz rho theta_v, computed on the
 * device with a fixed-order two-level reduction (bitwise reproducible);
 * synchronous.  The flux form keeps both constant to round-off (the
 * conservation invariants of the substep; the paper states none).  Either
 * output may be NULL.  Errors: ESTATE before a state is initialised, EHIP. */
int nhdc_diag(nhdc_ctx *ctx, double *mass, double *rho_theta, void *stream);

/* NHDC_EUNSTABLE if any prognostic value is NaN or Inf, else NHDC_OK; synchronous. */
int nhdc_check_finite(nhdc_ctx *ctx, void *stream);

/* Number of cells, edges, vertices and levels of the uploaded grid. */
int nhdc_sizes(const nhdc_ctx *ctx, int64_t *n_cells, int64_t *n_edges, int64_t *n_verts,
               int32_t *n_lev);

/* Level tiles of the marching kernels: each lane handles lt levels of one
 * entity (0 = the whole column).  Results do not depend on the tiles; only
 * speed does.  Edge kernels, the cell tendency kernel and the vertex kernel
 * are tiled separately.  nhdc_upload_grid (and nhdc_batch_create, over all
 * its instances) picks the starting shapes by size: each kind takes the
 * largest tile of whole, 48, 32, 16, 8 and 4 levels that gives it at least
 * 1024 blocks (4 per compute unit), and up to 40960 cells the column runs
 * its level-parallel build (NHDC_COLUMN_LEVELS); a streaming column with
 * fewer than 1024 blocks of 256 lanes runs in blocks of 64.  Grids of R2B6
 * (327680 cells) and larger start in whole columns with the streaming
 * column in blocks of 256.  The calls below override them. */
int nhdc_set_tiles(nhdc_ctx *ctx, int lt_edge, int lt_cell, int lt_vert);

/* Block shapes: the block sizes (lanes per workgroup: 64, 128 or 256) of the
 * column and the vertex kernels, the kernels whose work needs no per-block
 * tables (the others run in blocks of 256), and column_waves, the waves per
 * SIMD the column kernel may occupy (2 or 3, reserved through LDS; 0 = as
 * many as its registers allow, 4).  The defaults are 256, 64 and 3 (fewer
 * columns in flight keep more of the solve's scratch round trip in the
 * caches).  Results do not
 * depend on them; only speed does.  EINVAL for another value, ESTATE before
 * nhdc_upload_grid. */
int nhdc_set_block_sizes(nhdc_ctx *ctx, int column, int vertex, int column_waves);

/* Column solver build (the implicit vertical solve of Sec. 2, run by the
 * column kernels of both the predictor and the corrector):
 *   NHDC_COLUMN_STREAM (the default above 40960 cells): one lane per column marches down its
 *     levels forming the explicit parts and the Thomas factors, then back up
 *     with the back substitution and the level updates; the factors and the
 *     explicit parts of every level go to device memory in between.
 *   NHDC_COLUMN_LEVELS (the default up to 40960 cells): the levels of a
 *     column are shared among the lanes of a block (16 columns per block of
 *     256 lanes, 8 from 200 levels on); the lanes form their levels' explicit
 *     parts and tridiagonal rows in parallel into LDS, two lanes per column
 *     run the Thomas recurrence and the back substitution there, and the
 *     lanes apply their levels' updates in parallel.  For small shares of the
 *     GPU, where one lane's march down a whole column sets the step time.
 * Both give the same results to the bit (the same values formed by the same
 * operations in the same order); only speed differs.  EINVAL for another
 * mode, ESTATE before nhdc_upload_grid. */
#define NHDC_COLUMN_STREAM 0
#define NHDC_COLUMN_LEVELS 1
int nhdc_set_column_mode(nhdc_ctx *ctx, int mode);

/* The shapes the context's launches use now, into shapes[7] = {lt_edge,
 * lt_cell, lt_vert, block_column, block_vertex, column_waves, column_mode}:
 * the starting shapes of nhdc_upload_grid, or what the setters or the
 * autotuner chose since.  ESTATE before nhdc_upload_grid. */
int nhdc_get_shapes(const nhdc_ctx *ctx, int *shapes);

/* The autotuner (the paper tunes its GPU kernels per configuration, Sec.
 * 3.2; here a search the library runs itself): a coordinate search over the
 * level tiles, the block sizes and the column mode of this context's grid,
 * each candidate timed over whole steps of (dt, nsubsteps) on `stream`;
 * keeps the fastest and reports it in best[8] = {lt_edge, lt_cell, lt_vert,
 * block_column, block_vertex, column_waves, ms per step, column_mode} (the
 * caller provides 8 doubles).  The state is saved before and restored after
 * the search.  If cache_path is not NULL it names a JSON file (object of
 * "key": [lt_edge, lt_cell, lt_vert, block_column, block_vertex, column_waves,
 * ms, column_mode], the key naming the precision, the launch path and the
 * instances' shapes) that is read first (a hit skips the search) and updated
 * after a search. */
int nhdc_autotune(nhdc_ctx *ctx, double dt, int nsubsteps, const char *cache_path,
                  double *best, void *stream);

/* ---- batching -------------------------------------------------------------
 * A batch advances many independent instances (contexts with their grid and
 * state) of uneven size and level count together: every kernel of a substep
 * is ONE launch over all instances (the block map assigns each instance its
 * own range of tiles), and a whole step (nsubsteps x 10 launches) is captured
 * once into a HIP graph and replayed.  The paper's GPU runs keep small
 * kernels from starving the device with CUDA graphs (Sec. 3.1) and lose
 * efficiency when a GPU's share of the grid is small (Sec. 5); batching is
 * the single-GPU answer to both.  Instances keep their own dt; results are
 * bitwise those of stepping each instance alone with the same tiles. */
typedef struct nhdc_batch nhdc_batch;

#define NHDC_MAX_INST 64

/* Borrow n (1..NHDC_MAX_INST) contexts, all on one device and of one
 * precision, each with grid and state.  A context destroyed while a batch
 * holds it keeps its device memory, and keeps stepping in the batch, until
 * the last batch holding it is destroyed (the caller must not use the
 * context's handle after nhdc_destroy).  NHDC_EINVAL for n out of range, a
 * repeated context, or mixed devices or precisions; NHDC_ESTATE for a
 * context without grid or state, or destroyed while another batch holds it. */
int nhdc_batch_create(nhdc_batch **out, nhdc_ctx *const *instances, int n);
/* nsteps steps of (dt[i], nsubsteps) for every instance i, enqueued on stream. */
int nhdc_batch_step(nhdc_batch *b, const double *dt, int nsubsteps, int nsteps, void *stream);
int nhdc_batch_set_tiles(nhdc_batch *b, int lt_edge, int lt_cell, int lt_vert);
/* As nhdc_set_block_sizes, for the batch's launches (not the persistent one). */
int nhdc_batch_set_block_sizes(nhdc_batch *b, int column, int vertex, int column_waves);
/* As nhdc_set_column_mode, for the batch's launches (the persistent launch
 * runs the streaming build). */
int nhdc_batch_set_column_mode(nhdc_batch *b, int mode);
/* As nhdc_get_shapes, for the batch's launches. */
int nhdc_batch_get_shapes(const nhdc_batch *b, int *shapes);
/* Persistent form (on = 1): each step's substeps run as ONE cooperative
 * launch over every instance, with as many blocks as the GPU holds at once
 * (blocks_per_cu > 0 caps the blocks per compute unit below that); its
 * blocks take each phase's tiles in turn and a grid barrier separates the
 * phases.  The options' once-per-step work (diffusion, tracers) runs as
 * launches around it.  Results are bitwise those of the graph of launches.
 * on = 0 returns to the graph of launches.  EINVAL when an instance's
 * numbering leaves an edge block with more distinct cells than lanes or
 * without cell_vt's block tables (the persistent kernel is built for the
 * numbering along the curve), or without cooperative launch. */
int nhdc_batch_set_persistent(nhdc_batch *b, int on, int blocks_per_cu);
/* Blocks of the persistent launch (0 when the batch is not persistent). */
int nhdc_batch_persistent_grid(const nhdc_batch *b);
/* As nhdc_autotune, over the whole batch, on its current path (the
 * persistent path searches the level tiles only). */
int nhdc_batch_autotune(nhdc_batch *b, const double *dt, int nsubsteps, const char *cache_path,
                        double *best, void *stream);
const char *nhdc_batch_last_error(const nhdc_batch *b);
void nhdc_batch_destroy(nhdc_batch *b);

/* Per-kernel timing (the paper times with a cycle counter and reports the
 * dynamical core's sustained bandwidth, Sec. 3.2 and 4.3).  While enabled,
 * every kernel launch of nhdc_step is bracketed by HIP events on the step's
 * stream and nhdc_step synchronises that stream before returning, so the
 * timed work is the same kernels with events in between.  Enabling resets
 * the accumulators. */
int nhdc_set_timing(nhdc_ctx *ctx, int enable);
/* Number of distinct kernels reported by nhdc_kernel_stats. */
int nhdc_kernel_count(void);
/* Name, accumulated time [ms] and launch count of kernel `index` since timing
 * was enabled; NHDC_EINVAL for an index out of range. *name is static storage. */
int nhdc_kernel_stats(const nhdc_ctx *ctx, int index, const char **name, double *total_ms,
                      int64_t *launches);

/* ---- allocation-free entry point ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * global sums as nhdc_diag (dry mass sum A_c dz rho and sum A_c dz rho theta_v,
 * with the same fixed-order two-level reduction, so bitwise equal to it), over
 * caller-held device arrays, with no context and no allocation:
 *   cell_area [n_cells], zh [n_lev+1][n_cells] (half-level heights),
 *   rho, theta_v [n_lev][n_cells]: device memory, read only;
 *   out [2]: device memory, receives {mass, rho_theta}.
 * Asynchronous: the work is enqueued on `stream` (of the current device) and
 * out holds the sums once the stream reaches it; no synchronisation, host
 * copy, memset or allocation happens, so the call can be captured in a graph.
 * The per-block partials live in a fixed device array of the library
 * (2 doubles per 256 cells, NHDC_NOALLOC_MAX_CELLS cells at most: 1 MiB),
 * one per GPU, held until the process ends and shared by every call on that
 * GPU: calls that overlap on one GPU (different streams or threads) race;
 * calls ordered on one stream do not.  Every partial is written by the call
 * before it is read, so nothing carries over between calls.
 * Errors: NHDC_EINVAL for a NULL array, n_cells < 1 or n_lev outside
 * 1..NHDC_MAX_LEV; NHDC_ETOOBIG for n_cells > NHDC_NOALLOC_MAX_CELLS; NHDC_EHIP
 * when the launch fails.  nhdc_last_error(NULL) gives the calling thread's
 * message of the last failed call. */
#define NHDC_NOALLOC_MAX_CELLS (65536LL * 256)
int nhdc_diag_noalloc(int64_t n_cells, int32_t n_lev, const double *cell_area, const double *zh,
                      const double *rho, const double *theta_v, double *out, void *stream);

/* Message of the context's last failure; with ctx NULL, the calling thread's
 * last failure of a context-free call (nhdc_diag_noalloc). */
const char *nhdc_last_error(const nhdc_ctx *ctx);
/* Releases the context and its device memory; a context that a batch still
 * holds is released by the last nhdc_batch_destroy instead. */
void nhdc_destroy(nhdc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
