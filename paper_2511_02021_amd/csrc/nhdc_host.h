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

// The shapes a launch set starts with, by its size (host side only: they
// choose among the kernels' builds and block maps).  A share too small to
// fill the GPU with one lane per column spends its step waiting on one level
// after another: each marching kind then takes the largest level tile (of
// whole, 48, 32, 16, 8 and 4 levels) that gives it at least kFillBlocks
// blocks over all instances, and up to kSmallShare cells the column runs its
// level-parallel build.  A streaming column with fewer than kFillBlocks
// blocks of 256 lanes runs in blocks of 64, so that its few wavefronts spread
// over every CU.  Measured on 90-level grids in FP64, ms per step with whole
// columns -> these shapes: R2B3 (5120 cells) 5.9 -> 0.94, R2B4 (20480) 6.8 ->
// 3.0, R2B5 (81920) 10.6 -> 8.9; R2B6 and larger start in whole columns with
// the streaming column in blocks of 256, their best.
constexpr int64_t kFillBlocks = 1024;  // 256 CUs x 4 blocks
constexpr int64_t kSmallShare = 40960;
inline int fill_tile(const Grid *const *grids, int n, int kind_entities, int block) {
    const int cand[] = {0, 48, 32, 16, 8, 4};
    for (int lt : cand) {
        int64_t blocks = 0;
        for (int i = 0; i < n; ++i) {
            const Grid &g = *grids[i];
            const int64_t ent = kind_entities == 0 ? g.ne : kind_entities == 1 ? g.nc : g.nv;
            const int l = lt > 0 && lt < g.N ? lt : g.N;
            blocks += (ent + block - 1) / block * ((g.N + l - 1) / l);
        }
        if (blocks >= kFillBlocks) return lt;
    }
    return 4;
}
inline Tune default_tune(const Grid *const *grids, int n) {
    Tune t;
    int64_t cells = 0;
    for (int i = 0; i < n; ++i) cells += grids[i]->nc;
    t.lt_edge = fill_tile(grids, n, 0, BLOCK);
    t.lt_cell = fill_tile(grids, n, 1, BLOCK);
    t.lt_vert = fill_tile(grids, n, 2, t.blk_vert);
    t.col_mode = cells <= kSmallShare ? 1 : 0;
    if (t.col_mode == 0 && (cells + BLOCK - 1) / BLOCK < kFillBlocks) t.blk_col = 64;
    return t;
}
// shapes[7] of nhdc_get_shapes: lt_edge, lt_cell, lt_vert, block_column,
// block_vertex, column_waves, column_mode
inline void tune_shapes(const Tune &t, int *out) {
    const int v[7] = {t.lt_edge, t.lt_cell, t.lt_vert, t.blk_col, t.blk_vert, t.col_waves, t.col_mode};
    for (int i = 0; i < 7; ++i) out[i] = v[i];
}

}  // namespace nhdc
