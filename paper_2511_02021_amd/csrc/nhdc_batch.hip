// nhdc_batch.hip -- many independent instances advanced together: one launch
// per kernel over all instances, a whole step captured once into a HIP graph
// and replayed, level tiles from the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "nhdc_host.h"
#include "nhdc_internal.h"

using namespace nhdc;

struct nhdc_batch {
    int device = 0;
    std::vector<nhdc_ctx *> ctxs;
    Launcher L;
    Tune tune;
    hipStream_t cap = nullptr;          // private stream used only for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> graph_dt;       // the step the graph holds
    int graph_nsub = 0;
    Tune graph_tune;
    // persistent form: the substeps of a step as one cooperative launch
    bool persistent = false;
    PMaps *d_pm = nullptr;  // the maps in device memory (block size BLOCK for every kind)
    int grid = 0;           // blocks of the persistent launch
    std::string err;
};

namespace {

void drop_graph(nhdc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_dt.clear();
}

// The persistent launch's maps: the batch's level tiles, every kind in
// blocks of BLOCK lanes (the one block size of the persistent kernel).
int upload_pmaps(nhdc_batch *b, const Tune &t) {
    Tune tp = t;
    tp.blk_col = tp.blk_vert = BLOCK;
    tp.col_mode = 0;  // the persistent kernel runs the streaming column
    Launcher tmp;
    rebuild_maps(tmp, b->ctxs, tp);
    PMaps h;
    for (int k = 0; k < KIND_NUM; ++k) {
        h.maps[k] = tmp.maps[k];
        h.nblocks[k] = tmp.nblocks[k];
    }
    if (!b->d_pm) {
        b->d_pm = static_cast<PMaps *>(dev_alloc(b->L.al, sizeof(PMaps)));
        if (!b->d_pm) return set_err(b->err, NHDC_ENOMEM, "batch: persistent maps: allocation failed");
    }
    hipError_t e = hipStreamSynchronize(b->cap);
    if (e == hipSuccess) e = hipDeviceSynchronize();  // no launch may still read the old maps
    if (e == hipSuccess) e = hipMemcpy(b->d_pm, &h, sizeof(PMaps), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: persistent maps");
    return NHDC_OK;
}

bool graph_matches(const nhdc_batch *b, const double *dt, int nsub) {
    if (!b->exec || b->graph_nsub != nsub) return false;
    if (!same_tune(b->graph_tune, b->tune)) return false;  // tiles, block sizes, column mode
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (b->graph_dt[i] != dt[i]) return false;
    return true;
}

// Capture one step (nsub substeps x 10 launches over all instances) into a graph.
int capture(nhdc_batch *b, const double *dt, int nsub) {
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipStreamBeginCapture");
    hipError_t le = run_step(b->L, dt, nsub, nullptr, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(b->err, le, "batch: launch during capture");
    }
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_fail(b->err, e, "batch: hipGraphInstantiate");
    }
    b->graph_dt.assign(dt, dt + b->ctxs.size());
    b->graph_nsub = nsub;
    b->graph_tune = b->tune;
    return NHDC_OK;
}

int check_dt(nhdc_batch *b, const double *dt, int nsub) {
    if (!dt) return set_err(b->err, NHDC_EINVAL, "batch: dt is NULL");
    if (nsub < 1) return set_err(b->err, NHDC_EINVAL, "batch: nsubsteps must be >= 1");
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (!(dt[i] > 0) || !std::isfinite(dt[i]))
            return set_err(b->err, NHDC_EINVAL, "batch: dt must be positive and finite");
    return NHDC_OK;
}

}  // namespace

extern "C" {

int nhdc_batch_create(nhdc_batch **out, nhdc_ctx *const *inst, int n) {
    if (!out) return NHDC_EINVAL;
    *out = nullptr;
    if (!inst || n < 1 || n > MAX_INST) return NHDC_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!inst[i] || !inst[i]->grid_ready || !inst[i]->state_ready || inst[i]->destroy_pending)
            return NHDC_ESTATE;
        if (inst[i]->device != inst[0]->device || inst[i]->precision != inst[0]->precision)
            return NHDC_EINVAL;
        for (int j = 0; j < i; ++j)
            if (inst[j] == inst[i]) return NHDC_EINVAL;  // each instance once
    }
    nhdc_batch *b = new (std::nothrow) nhdc_batch;
    if (!b) return NHDC_ENOMEM;
    b->device = inst[0]->device;
    b->ctxs.assign(inst, inst + n);
    b->L.al = inst[0]->al;  // the batch's descriptors come from its first instance's allocator
    if (hipSetDevice(b->device) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return NHDC_EHIP;
    }
    if (upload_insts(b->L, b->ctxs, b->err) != NHDC_OK) {
        (void)hipStreamDestroy(b->cap);
        delete b;
        return NHDC_ENOMEM;
    }
    std::vector<const Grid *> grids;
    for (auto *c : b->ctxs) grids.push_back(&c->g);
    b->tune = default_tune(grids.data(), int(grids.size()));
    rebuild_maps(b->L, b->ctxs, b->tune);
    for (auto *c : b->ctxs) ++c->in_batches;
    *out = b;
    return NHDC_OK;
}

int nhdc_batch_step(nhdc_batch *b, const double *dt, int nsub, int nsteps, void *stream) {
    if (!b) return NHDC_EINVAL;
    int rc = check_dt(b, dt, nsub);
    if (rc) return rc;
    if (nsteps < 0) return set_err(b->err, NHDC_EINVAL, "batch: nsteps must be >= 0");
    if (hipSetDevice(b->device) != hipSuccess) return set_err(b->err, NHDC_EHIP, "batch: hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->persistent) {
        for (int i = 0; i < nsteps; ++i) {
            hipError_t e = run_step_persistent(b->L, b->d_pm, b->grid, dt, nsub, s);
            if (e != hipSuccess) return hip_fail(b->err, e, "batch: persistent launch");
        }
        return NHDC_OK;
    }
    if (!graph_matches(b, dt, nsub) && (rc = capture(b, dt, nsub))) return rc;
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(b->err, e, "batch: hipGraphLaunch");
    }
    return NHDC_OK;
}

int nhdc_batch_set_tiles(nhdc_batch *b, int lt_edge, int lt_cell, int lt_vert) {
    if (!b) return NHDC_EINVAL;
    if (lt_edge < 0 || lt_cell < 0 || lt_vert < 0)
        return set_err(b->err, NHDC_EINVAL, "batch: tiles must be >= 0");
    b->tune.lt_edge = lt_edge;
    b->tune.lt_cell = lt_cell;
    b->tune.lt_vert = lt_vert;
    rebuild_maps(b->L, b->ctxs, b->tune);
    return b->persistent ? upload_pmaps(b, b->tune) : NHDC_OK;
}

int nhdc_batch_set_block_sizes(nhdc_batch *b, int column, int vertex, int column_waves) {
    if (!b) return NHDC_EINVAL;
    if (!valid_block(column) || !valid_block(vertex) || !valid_waves(column_waves))
        return set_err(b->err, NHDC_EINVAL,
                       "batch: block sizes must be 64, 128 or 256 and column_waves 0, 2 or 3");
    b->tune.blk_col = column;
    b->tune.blk_vert = vertex;
    b->tune.col_waves = column_waves;
    rebuild_maps(b->L, b->ctxs, b->tune);
    return NHDC_OK;
}

int nhdc_batch_set_column_mode(nhdc_batch *b, int mode) {
    if (!b) return NHDC_EINVAL;
    if (!valid_col_mode(mode))
        return set_err(b->err, NHDC_EINVAL, "batch: column mode must be 0 (stream) or 1 (levels)");
    b->tune.col_mode = mode;
    rebuild_maps(b->L, b->ctxs, b->tune);
    return NHDC_OK;
}

int nhdc_batch_get_shapes(const nhdc_batch *b, int *shapes) {
    if (!b || !shapes) return NHDC_EINVAL;
    tune_shapes(b->tune, shapes);
    return NHDC_OK;
}

int nhdc_batch_set_persistent(nhdc_batch *b, int on, int blocks_per_cu) {
    if (!b) return NHDC_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return set_err(b->err, NHDC_EHIP, "batch: hipSetDevice");
    if (!on) {
        b->persistent = false;
        return NHDC_OK;
    }
    if (blocks_per_cu < 0) return set_err(b->err, NHDC_EINVAL, "batch: blocks_per_cu must be >= 0");
    if (b->L.vt_two || !b->L.cvt_lds)
        return set_err(b->err, NHDC_EINVAL,
                       "batch: the persistent form needs every instance numbered along the curve "
                       "(edge blocks with at most one distinct cell per lane and cell_vt's block tables)");
    int coop = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, b->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess)
        e = form_ops(b->L.precision).persistent_blocks(b->L, &per_cu);
    if (e != hipSuccess) return hip_fail(b->err, e, "batch: persistent launch properties");
    if (!coop || per_cu < 1) return set_err(b->err, NHDC_EINVAL, "batch: no cooperative launch on this device");
    const int use = blocks_per_cu > 0 && blocks_per_cu < per_cu ? blocks_per_cu : per_cu;
    int rc = upload_pmaps(b, b->tune);
    if (rc) return rc;
    b->grid = use * ncu;
    b->persistent = true;
    return NHDC_OK;
}

int nhdc_batch_persistent_grid(const nhdc_batch *b) { return b && b->persistent ? b->grid : 0; }

int nhdc_batch_autotune(nhdc_batch *b, const double *dt, int nsub, const char *cache_path,
                        double *best, void *stream) {
    if (!b) return NHDC_EINVAL;
    int rc = check_dt(b, dt, nsub);
    if (rc) return rc;
    if (hipSetDevice(b->device) != hipSuccess) return set_err(b->err, NHDC_EHIP, "batch: hipSetDevice");
    drop_graph(b);
    Stepper stepper;
    if (b->persistent) {
        // the persistent kernel runs every kind in blocks of BLOCK lanes:
        // only the level tiles are searched
        stepper.block_sizes = false;
        stepper.prepare = [b](const Tune &t) -> hipError_t {
            return upload_pmaps(b, t) == NHDC_OK ? hipSuccess : hipErrorUnknown;
        };
        stepper.step = [b](const double *d, int ns, hipStream_t st) {
            return run_step_persistent(b->L, b->d_pm, b->grid, d, ns, st);
        };
    } else {
        const Launcher &L = b->L;
        stepper.step = [&L](const double *d, int ns, hipStream_t st) { return run_step(L, d, ns, nullptr, st); };
    }
    return autotune(b->L, b->tune, b->ctxs, dt, nsub, cache_path, best,
                    static_cast<hipStream_t>(stream), b->err, stepper,
                    b->persistent ? "persistent" : "launches");
}

const char *nhdc_batch_last_error(const nhdc_batch *b) { return b ? b->err.c_str() : "no batch"; }

void nhdc_batch_destroy(nhdc_batch *b) {
    if (!b) return;
    if (hipSetDevice(b->device) == hipSuccess) {
        (void)hipDeviceSynchronize();  // replays still in flight read the descriptors
        drop_graph(b);
        dev_free(b->L.al, b->L.d_insts);
        dev_free(b->L.al, b->d_pm);
        if (b->cap) (void)hipStreamDestroy(b->cap);
    }
    for (auto *c : b->ctxs) {
        --c->in_batches;
        if (c->in_batches == 0 && c->destroy_pending) free_context(c);
    }
    delete b;
}

}  // extern "C"
