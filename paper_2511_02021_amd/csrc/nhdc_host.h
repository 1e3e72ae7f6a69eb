// nhdc_host.h -- host helpers shared by contexts and batches.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "nhdc_internal.h"

namespace nhdc {
int set_err(std::string &err, int code, const std::string &msg);
int hip_fail(std::string &err, hipError_t e, const char *where);
// enqueue one step (nsub substeps) of every instance of L; dt[i] per instance
hipError_t run_step(const Launcher &L, const double *dt, int nsub, Timing *tm, hipStream_t st);
// enqueue one step of every instance of L with its substeps as one
// persistent cooperative launch of `grid` blocks over the maps d_pm
hipError_t run_step_persistent(const Launcher &L, const PMaps *d_pm, int grid, const double *dt,
                               int nsub, hipStream_t st);
void rebuild_maps(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, const Tune &t);
int upload_insts(Launcher &L, const std::vector<nhdc_ctx *> &ctxs, std::string &err);
// How the autotuner runs a candidate: prepare (after the maps are rebuilt
// for its tiles and block sizes; may be empty) and one step; block_sizes:
// whether the path takes the column and vertex block sizes.
struct Stepper {
    std::function<hipError_t(const Tune &)> prepare;
    std::function<hipError_t(const double *, int, hipStream_t)> step;
    bool block_sizes = true;
};
// Coordinate search of the column mode, the tiles and the block sizes (the
// tiles alone when the stepper takes no block sizes) by timing whole steps
// on a snapshot of the state, restored afterwards; best_out[8] = {lt_edge,
// lt_cell, lt_vert, block_column, block_vertex, column_waves, ms,
// column_mode}; the JSON cache is keyed by precision, path_tag and the
// instances' shapes.
int autotune(Launcher &L, Tune &tune, const std::vector<nhdc_ctx *> &ctxs, const double *dt,
             int nsub, const char *cache_path, double *best_out, hipStream_t st,
             std::string &err, const Stepper &stepper, const char *path_tag);
// shapes[7] of nhdc_get_shapes: lt_edge, lt_cell, lt_vert, block_column,
// block_vertex, column_waves, column_mode
inline void tune_shapes(const Tune &t, int *out) {
    const int v[7] = {t.lt_edge, t.lt_cell, t.lt_vert, t.blk_col, t.blk_vert, t.col_waves, t.col_mode};
    for (int i = 0; i < 7; ++i) out[i] = v[i];
}

}  // namespace nhdc
